// Device kernels of the oMAP planner for gfx950 (CDNA4, wave64).
//
// The network of the paper (Sec. Methods, "Activity Map Generation"; Fig. net)
// applies L identical layers  A <- ReLU(maxpool3x3(A) + I_e + I_s)  starting
// from A_0 = I_s.  The kernels run the same layers in an integer encoding with
// a per-layer decrement: V_0 = K at the sources and 0 elsewhere, and
//     V'(x) = 0                                   x an obstacle
//     V'(x) = max(V(x), max over the 3x3 window of V - 1)   otherwise
// With K = L + 1 the fixpoint of this update equals A_L exactly (both are
// max(0, L + 1 - d(x)) with d the 8-neighbour step distance to the nearest
// source), it is reached after at most L sweeps, and further sweeps leave it
// unchanged.  Because the update is monotone and bounded by that fixpoint, any
// schedule of tile updates that keeps visiting tiles whose neighbourhood
// changed reaches the same bits; the tests compare against the paper's literal
// layers.  With K = 2^31 - 1 the fixpoint is K - d and the run-time determined
// layer count L* is K minus the smallest positive value.
//
// In registers an obstacle is the value 0x80000000 (the sign bit).  Signed
// max-pooling ignores it; the update  max_u32(V, sat_sub_u32(m, 1))  keeps it
// (0x80000000 is above any activity as unsigned) and clamps free cells at 0,
// so one unsigned max and one saturating subtract implement decrement, ReLU and
// obstacle masking together.

#include "omap_internal.h"

namespace omap {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int max3i(int a, int b, int c) { return max(max(a, b), c); }

__device__ __forceinline__ uint32_t sat_dec(uint32_t x) {
    return __builtin_elementwise_sub_sat(x, 1u);
}

// Lane l receives lane l-1's value (DPP wave_shr:1).  Lane 0 has no source
// and reads 0; the kernels only use that lane's result inside the halo.
__device__ __forceinline__ int from_left_lane(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);
}

// Lane l receives lane l+1's value (DPP wave_shl:1); lane 63 reads 0.
__device__ __forceinline__ int from_right_lane(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kLanes - 1); }

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

__global__ void k_fill(int32_t* __restrict__ p, int64_t n4, int32_t value) {
    int4 v = make_int4(value, value, value, value);
    int4* q = reinterpret_cast<int4*>(p);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        q[i] = v;
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

__device__ __forceinline__ int64_t tile_cells(const MazeDev& md, int ty, int tx, int tile_rows,
                                              int tile_cols) {
    return (int64_t)min(tile_rows, md.H - ty * tile_rows) * min(tile_cols, md.W - tx * tile_cols);
}

// Append tile (ty, tx) of `slot` to a.list_out unless it is already there
// (flag exchange) and count it in the slot's scheduled tiles.  One lane.
__device__ __forceinline__ void schedule_tile(const RoundArgs& a, const MazeDev& md, int slot, int ty,
                                              int tx) {
    const int g = md.tile_base + ty * md.tiles_x + tx;
    if (atomicExch(&a.flags_out[g], 1) == 0) {
        const int k = atomicAdd(a.count_out, 1);
        a.list_out[2 * k] = g;
        a.list_out[2 * k + 1] = slot;
        if (a.n_slots > 1) atomicAdd(&a.sched_out[slot], 1);
    }
}

// The same for the 3x3 tiles around (ty, tx), from a whole wave: lanes 0..8
// claim one tile each, then a single atomic reserves the list entries of all
// the lanes that won their claim.
__device__ __forceinline__ void schedule_neighbourhood(const RoundArgs& a, const MazeDev& md, int slot,
                                                       int ty, int tx) {
    const int lane = lane_id();
    const int ny = ty + lane / 3 - 1, nx = tx + lane % 3 - 1;
    const int g = md.tile_base + ny * md.tiles_x + nx;
    bool won = false;
    if (lane < 9 && ny >= 0 && ny < md.tiles_y && nx >= 0 && nx < md.tiles_x)
        won = atomicExch(&a.flags_out[g], 1) == 0;
    const uint64_t mask = __ballot(won);
    if (mask == 0) return;
    const int n = __popcll(mask);
    int base = 0;
    if (lane == 0) {
        base = atomicAdd(a.count_out, n);
        if (a.n_slots > 1) atomicAdd(&a.sched_out[slot], n);
    }
    base = __builtin_amdgcn_readfirstlane(base);
    if (won) {
        const int k = base + __popcll(mask & ((1ull << lane) - 1));
        a.list_out[2 * k] = g;
        a.list_out[2 * k + 1] = slot;
    }
}

// Pushes one tile, already counted as pending, onto the asynchronous work
// queue (see k_sweep_async).  One lane.
__device__ __forceinline__ void queue_push(const AsyncQueue& q, int g, int slot) {
    const uint32_t k = atomicAdd(q.tail, 1u);
    const unsigned long long e = ((unsigned long long)(uint32_t)slot << 32) | (uint32_t)(g + 1);
    if (atomicCAS(q.ring + (k & q.ring_mask), 0ull, e) != 0ull) atomicAdd(q.error, 1);
}

// Seed V := K at the sources (both buffers) and, when `schedule` is set,
// schedule the tiles whose interior or halo holds a source.
__global__ void k_seed(RoundArgs a, int32_t slot, const int32_t* __restrict__ src, int32_t n,
                       int32_t schedule, int32_t* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
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
    const int ty = r / a.tile_rows, tx = c / a.tile_cols;
    a.touched[md.tile_base + ty * md.tiles_x + tx] = 1;
    if (!schedule) return;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int ny = ty + dy, nx = tx + dx;
            if (ny < 0 || ny >= md.tiles_y || nx < 0 || nx >= md.tiles_x) continue;
            if (a.async) {
                const int g = md.tile_base + ny * md.tiles_x + nx;
                if (atomicOr(&a.q.state[g], 1) == 0 && atomicAdd(a.q.pending, 1) >= 0) queue_push(a.q, g, slot);
            } else {
                schedule_tile(a, md, slot, ny, nx);
            }
        }
}

// ---------------------------------------------------------------------------
// the sweep: T layers per tile visit, one wave per tile
// ---------------------------------------------------------------------------
//
// A tile is `rows` x TW interior cells (TW = 256 - 2T) at (r0, c0).  The wave
// streams the 256-column strip [c0 - T, c0 - T + 256) from row r0 - T down to
// row r0 + rows + T - 1; lane l holds columns c0 - T + 4l .. +3.  Stage s of
// a T-stage register pipeline applies layer s+1 to the rows stage s-1 emits,
// one row behind it, keeping its last two input rows in registers.  Cells
// within s of the strip's edges after s layers are wrong (their neighbours
// were not loaded), and that region is exactly the halo; the interior is exact
// after T layers (trapezoidal temporal blocking).  Out-of-grid positions load
// as obstacles, which is the zero padding of the paper's pooling.

// One row step of the pipeline (C columns per lane).  Stage s keeps its last
// three input rows in st[s][0..2]; on the step with P = i mod 3 the newest row
// (i) sits in slot P, row i-1 in slot (P+2) mod 3 and row i-2 in slot
// (P+1) mod 3.  Stage s writes its output row straight into stage s+1's slot
// P, whose previous content (row i-3 of that stage) is dead, so no register
// copies are needed.
// With GUARD, stages above smax are skipped (see sweep_tile).
template <int T, int P, int C, bool GUARD>
__device__ __forceinline__ void sweep_row(uint32_t (&st)[T][3][C], uint32_t (&out)[C], int smax) {
    constexpr int PA = (P + 1) % 3, PB = (P + 2) % 3;
#pragma unroll
    for (int s = 0; s < T; ++s) {
        if (!GUARD || s <= smax) {
            const uint32_t* a = st[s][PA];   // row above the centre
            const uint32_t* b = st[s][PB];   // centre row
            const uint32_t* c = st[s][P];    // row below the centre
            int v[C];
#pragma unroll
            for (int j = 0; j < C; ++j) v[j] = max3i((int)a[j], (int)b[j], (int)c[j]);
            const int left = from_left_lane(v[C - 1]);
            const int right = from_right_lane(v[0]);
            uint32_t* o = (s + 1 < T) ? st[s + 1 < T ? s + 1 : s][P] : out;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const int l = j == 0 ? left : v[j - 1];
                const int r = j == C - 1 ? right : v[j + 1];
                o[j] = max(b[j], sat_dec((uint32_t)max3i(l, v[j], r)));
            }
        }
    }
}

// Global-memory views of the activity and mask buffers (lets the compiler use
// global_load / global_store instead of flat accesses).
typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef int v2i32 __attribute__((ext_vector_type(2)));
template <int C> struct LaneVec;
template <> struct LaneVec<4> { typedef v4i32 type; };
template <> struct LaneVec<2> { typedef v2i32 type; };
typedef const __attribute__((address_space(1))) uint32_t gconst_u32;

template <int C>
__device__ __forceinline__ typename LaneVec<C>::type gload(const int32_t* p) {
    typedef typename LaneVec<C>::type V;
    return *(const __attribute__((address_space(1))) V*)p;
}

template <int C>
__device__ __forceinline__ void gstore(int32_t* p, typename LaneVec<C>::type v) {
    typedef typename LaneVec<C>::type V;
    *(__attribute__((address_space(1))) V*)p = v;
}

// Issues the loads of row R of the strip: C activity values and the mask word
// holding their bits.  Rows and columns outside the grid are clamped to a valid
// address (the loads are unconditional, so they can stay in flight); the decode
// in sweep_iter turns them into obstacles.
template <int C>
__device__ __forceinline__ void load_row(const MazeDev& md, const int32_t* Vin, int R,
                                         int col, bool col_ok, typename LaneVec<C>::type& v,
                                         uint32_t& w) {
    const int Rc = min(max(R, 0), md.H - 1);
    const int cc = col_ok ? col : 0;
    v = gload<C>(Vin + (int64_t)Rc * md.pitch + cc);
    w = *(gconst_u32*)(md.mask + (int64_t)Rc * md.mpitch + (cc >> 5));
}

// One row of the tile.  (v, w) holds row R, loaded one group (three rows)
// earlier; it is decoded into stage 0's slot P (cells outside the grid become
// exactly 0x80000000) and the same registers then receive the load of row
// R + 3, whose latency overlaps the T-stage arithmetic of the next rows.
template <int T, int P, int C, bool GUARD>
__device__ __forceinline__ void sweep_iter(uint32_t (&st)[T][3][C], typename LaneVec<C>::type& v,
                                           uint32_t& w, const MazeDev& md,
                                           const int32_t* Vin, int32_t* Vout, int R, int r0, int r_end,
                                           int col, bool col_ok, bool inner, int smax,
                                           uint64_t& sum_in, uint64_t& sum_out) {
    const bool ok = R >= 0 && R < md.H && col_ok;
    const uint32_t keep = ok ? 0xffffffffu : 0u;
    const uint32_t bits = ok ? (w >> (col & 31)) : 0xFu;   // outside the grid: obstacle
    uint32_t* c = st[0][P];
#pragma unroll
    for (int j = 0; j < C; ++j) c[j] = ((uint32_t)v[j] & keep) | (((bits >> j) & 1u) << 31);
    load_row<C>(md, Vin, R + 3, col, col_ok, v, w);
    if (inner && R >= r0 && R < r_end) {
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) t += c[j] & 0x7fffffffu;
        sum_in += t;
    }
    uint32_t out[C] = {};   // left 0 when the last stage is skipped (its row is not stored then)
    sweep_row<T, P, C, GUARD>(st, out, smax);
    const int Ro = R - T;
    if (inner && Ro >= r0 && Ro < r_end) {
        typename LaneVec<C>::type o;
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            o[j] = (int)(out[j] & 0x7fffffffu);
            t += (uint32_t)o[j];
        }
        gstore<C>(Vout + (int64_t)Ro * md.pitch + col, o);
        sum_out += t;
    }
}

// Returns true (wave-uniform) if any interior cell of the tile changed.  The
// wave streams the strip of 64*C columns starting T columns left of the tile.
// In place (IN_PLACE) the tile reads and writes buffer `parity`: a row is
// stored only after it and the T rows below it were loaded, so the visit never
// reads its own output.
template <int T, int C, bool IN_PLACE = false>
__device__ bool sweep_tile(const MazeDev& md, int ty, int tx, int tile_rows, int parity) {
    constexpr int TW = kLanes * C - 2 * T;
    constexpr int HALO_LANES = T / C;
    const int lane = lane_id();
    const int r0 = ty * tile_rows;
    const int r_end = min(r0 + tile_rows, md.H);
    const int col = tx * TW - T + C * lane;
    const bool col_ok = col >= 0 && col < md.pitch;
    const bool inner = lane >= HALO_LANES && lane < kLanes - HALO_LANES && col < md.W;
    int32_t* const Vin = parity ? md.V[1] : md.V[0];
    int32_t* const Vout = IN_PLACE ? Vin : (parity ? md.V[0] : md.V[1]);

    uint32_t st[T][3][C];
#pragma unroll
    for (int s = 0; s < T; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < C; ++j) st[s][k][j] = kObstacleBit;

    uint64_t sum_in = 0, sum_out = 0;
    const int n_iter = (r_end - r0) + 2 * T;   // rows r0-T .. r_end+T-1
    typename LaneVec<C>::type v0, v1, v2;
    uint32_t w0, w1, w2;
    load_row<C>(md, Vin, r0 - T, col, col_ok, v0, w0);
    load_row<C>(md, Vin, r0 - T + 1, col, col_ok, v1, w1);
    load_row<C>(md, Vin, r0 - T + 2, col, col_ok, v2, w2);
    // Stage s at step i (input row r0 - T + i) emits row r0 - T + i - 1 - s
    // after s + 1 layers; the stored rows [r0, r_end) after T layers need
    // exactly the emissions with i >= 2s + 2 (each of which reads only
    // emissions of stage s - 1 with i - 2 >= 2(s - 1) + 2).  So during the
    // first 2T steps, stages s > i/2 - 1 are skipped: the top of the tile's
    // trapezoid, a third of the work of a tile with as many rows as layers.
    constexpr int kWarm = 3 * ((2 * T + 2) / 3);   // >= 2T, a multiple of 3
    int i = 0;
    for (; i < kWarm; i += 3) {
        const int R = r0 - T + i;
        sweep_iter<T, 0, C, true>(st, v0, w0, md, Vin, Vout, R, r0, r_end, col, col_ok, inner, (i >> 1) - 1,
                                  sum_in, sum_out);
        sweep_iter<T, 1, C, true>(st, v1, w1, md, Vin, Vout, R + 1, r0, r_end, col, col_ok, inner,
                                  ((i + 1) >> 1) - 1, sum_in, sum_out);
        sweep_iter<T, 2, C, true>(st, v2, w2, md, Vin, Vout, R + 2, r0, r_end, col, col_ok, inner,
                                  ((i + 2) >> 1) - 1, sum_in, sum_out);
    }
    for (; i < n_iter; i += 3) {
        const int R = r0 - T + i;
        sweep_iter<T, 0, C, false>(st, v0, w0, md, Vin, Vout, R, r0, r_end, col, col_ok, inner, 0, sum_in, sum_out);
        sweep_iter<T, 1, C, false>(st, v1, w1, md, Vin, Vout, R + 1, r0, r_end, col, col_ok, inner, 0, sum_in,
                                   sum_out);
        sweep_iter<T, 2, C, false>(st, v2, w2, md, Vin, Vout, R + 2, r0, r_end, col, col_ok, inner, 0, sum_in,
                                   sum_out);
    }
    return __ballot(sum_in != sum_out) != 0;
}

// Marks `slot` for its first round: counters cleared, last round = r - 1; in
// the dense schedule the maze is flagged as changed so round r visits it.
__global__ void k_slot_reset(RoundArgs a, int32_t slot) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    a.maze_last_round[slot] = a.round_id - 1;
    for (int k = 0; k < kSpread; ++k) {
        a.maze_visits[slot * kSpread + k] = 0;
        a.maze_cell_visits[slot * kSpread + k] = 0;
    }
    if (a.dense) a.dchg_prev[slot] = 1;
}

// Loads of scheduling data that another block may have written in an earlier
// round of the same (persistent) launch: agent-scope atomic loads bypass the
// per-CU caches.
__device__ __forceinline__ int32_t load_shared(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The same for an 8-byte-aligned pair of int32 (low word first).
__device__ __forceinline__ uint64_t load_shared64(const int32_t* p) {
    return __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Round r: every scheduled tile gets T layers.  Active schedule: the tiles of
// a.list_in; a changed tile schedules itself and its 8 neighbour tiles for
// round r+1.  Dense schedule: every tile of each maze that changed in round
// r-1; a changed tile flags its maze for round r+1.  Block 0 also clears the
// buffers round r+1 will fill.
template <int T, int C>
__device__ __forceinline__ void sweep_round(const RoundArgs& a) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = lane_id();
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) *a.count_clear = 0;
        for (int m = threadIdx.x; m < a.n_slots; m += blockDim.x) {
            a.sched_clear[m] = 0;
            a.dchg_clear[m] = 0;
        }
    }
    const int stride = gridDim.x * kWavesPerBlock;
    int i = blockIdx.x * kWavesPerBlock + wave;
    // the count and the first list entry are loaded together (the entry is in
    // bounds for any i below the tile id space, and used only if i < n)
    const int n = a.dense ? a.n_tile_ids : __builtin_amdgcn_readfirstlane(load_shared(a.count_in));
    uint64_t e = (!a.dense && i < a.n_tile_ids) ? load_shared64(a.list_in + 2 * i) : 0;
    for (; i < n; i += stride) {
        int g, slot;
        if (a.dense) {
            g = i;
            slot = a.tile_maze[g];
            if (slot < 0 || __builtin_amdgcn_readfirstlane(load_shared(a.dchg_prev + slot)) == 0) continue;
        } else {
            g = __builtin_amdgcn_readfirstlane((int)(uint32_t)e);
            slot = __builtin_amdgcn_readfirstlane((int)(uint32_t)(e >> 32));
            if (i + stride < n) e = load_shared64(a.list_in + 2 * (i + stride));
            if (lane == 0) a.flags_in[g] = 0;
        }
        const MazeDev md = a.mazes[slot];
        const int lt = g - md.tile_base;
        const int ty = lt / md.tiles_x;
        const int tx = lt - ty * md.tiles_x;
        if (lane == 0) {
            const unsigned long long cells =
                (unsigned long long)tile_cells(md, ty, tx, a.tile_rows, a.tile_cols);
            const int sp = blockIdx.x & (kSpread - 1);
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_visits[slot * kSpread + sp]), 1ull);
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_cell_visits[slot * kSpread + sp]), cells);
            atomicAdd(a.total_cells + sp, cells);
            if (a.maze_last_round[slot] != a.round_id) a.maze_last_round[slot] = a.round_id;
            a.touched[g] = 1;
        }
        if (sweep_tile<T, C>(md, ty, tx, a.tile_rows, a.parity)) {
            if (a.dense) {
                if (lane == 0) {
                    a.dchg_cur[slot] = 1;
                    *a.count_out = 1;
                }
            } else {
                schedule_neighbourhood(a, md, slot, ty, tx);
            }
        }
    }
}

template <int T, int C>
__global__ __launch_bounds__(kBlockThreads) void k_sweep(RoundArgs a) {
    sweep_round<T, C>(a);
}

// Device-wide barrier of a cooperative launch (all blocks resident): the last
// block to arrive resets the counter and advances the generation; the others
// wait for the generation to change.  Fences on both sides publish this
// block's writes and drop stale lines from the CU's caches.
__device__ __forceinline__ void grid_barrier(unsigned int* count, unsigned int* gen) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        if (atomicAdd(count, 1u) == gridDim.x - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(gen, 1u);
        } else {
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g)
                __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    __threadfence();
}

// Up to p.max_rounds rounds in one cooperative launch, stopping after the
// first round that schedules nothing (every resident maze converged).  The
// stop test reads the round's final count after the barrier, so every block
// takes the same decision.
template <int T, int C>
__global__ __launch_bounds__(kBlockThreads) void k_sweep_persistent(PersistentArgs p) {
    int k = 0;
    for (; k < p.max_rounds; ++k) {
        RoundArgs a = p.base;
        const int r = p.r0_mod6 + k;
        const int r2 = r & 1, r3 = r % 3, n3 = (r3 + 1) % 3, nn3 = (r3 + 2) % 3;
        const size_t cs = (size_t)p.base.n_slots;
        a.list_in = p.list[r2];
        a.count_in = p.count + r3;
        a.flags_in = p.flags[r2];
        a.list_out = p.list[r2 ^ 1];
        a.count_out = p.count + n3;
        a.flags_out = p.flags[r2 ^ 1];
        a.count_clear = p.count + nn3;
        a.sched_out = p.sched + n3 * cs;
        a.sched_clear = p.sched + nn3 * cs;
        a.dchg_prev = p.dchg + nn3 * cs;
        a.dchg_cur = p.dchg + r3 * cs;
        a.dchg_clear = p.dchg + n3 * cs;
        a.round_id = p.base.round_id + k;
        a.parity = r2;
        sweep_round<T, C>(a);
        grid_barrier(p.bar_count, p.bar_gen);
        if (load_shared(a.count_out) == 0) {
            ++k;
            break;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *p.rounds_done = k;
}

// ---------------------------------------------------------------------------
// asynchronous launch: a work queue instead of rounds
// ---------------------------------------------------------------------------
//
// Tiles are visited in place, in any order, by waves that take them from a
// ring of (slot, tile) entries.  A tile whose visit changed its interior marks
// itself and its 8 neighbour tiles as needing a visit: an idle tile is pushed,
// a tile being visited is flagged and pushed again when its visit ends (the
// values that visit read may predate the change).  Because the update is
// monotone and bounded by its fixpoint, values read while a neighbour is being
// written are lower bounds, every visit only raises values, and the launch
// reaches the same fixpoint bits as the round schedules once no tile needs a
// visit.  Agent-scope release / acquire fences order a tile's stores before
// the marks it makes and a visit's loads after the mark that queued it.

// Marks `slot`'s tiles around (ty, tx) (lanes 0..8, one tile each); idle tiles
// are counted as pending and pushed with one reservation for the whole wave.
__device__ __forceinline__ void queue_mark_neighbourhood(const AsyncQueue& q, const MazeDev& md, int slot,
                                                         int ty, int tx) {
    const int lane = lane_id();
    const int ny = ty + lane / 3 - 1, nx = tx + lane % 3 - 1;
    const int g = md.tile_base + ny * md.tiles_x + nx;
    bool won = false;
    if (lane < 9 && ny >= 0 && ny < md.tiles_y && nx >= 0 && nx < md.tiles_x)
        won = atomicOr(&q.state[g], 1) == 0;
    const uint64_t mask = __ballot(won);
    if (mask == 0) return;
    const int n = __popcll(mask);
    uint32_t base = 0;
    if (lane == 0) {
        // pending is raised before the entries can be taken: the second
        // atomic's operand depends on the first one's result (p >= 0 always)
        const int p = atomicAdd(q.pending, n);
        base = atomicAdd(q.tail, (uint32_t)n + (uint32_t)(p < 0));
    }
    base = __builtin_amdgcn_readfirstlane(base);
    if (won) {
        const uint32_t k = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1));
        const unsigned long long e = ((unsigned long long)(uint32_t)slot << 32) | (uint32_t)(g + 1);
        if (atomicCAS(q.ring + (k & q.ring_mask), 0ull, e) != 0ull) atomicAdd(q.error, 1);
    }
}

template <int T, int C>
__global__ __launch_bounds__(kBlockThreads) void k_sweep_async(RoundArgs a) {
    const AsyncQueue& q = a.q;
    const int lane = lane_id();
    const unsigned long long t0 = wall_clock64();
    for (;;) {
        if (wall_clock64() - t0 > q.budget) break;          // pause: the host relaunches
        uint32_t ticket = 0;
        if (lane == 0) ticket = atomicAdd(q.head, 1u);
        ticket = __builtin_amdgcn_readfirstlane(ticket);
        unsigned long long* ep = q.ring + (ticket & q.ring_mask);
        unsigned long long e = 0;
        for (int poll = 0;; ++poll) {
            e = __hip_atomic_load(ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            e = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(e >> 32)) << 32) |
                __builtin_amdgcn_readfirstlane((uint32_t)e);
            if (e != 0) break;
            if ((poll & 7) == 7 && (__builtin_amdgcn_readfirstlane(load_shared(q.done)) != 0 ||
                                    wall_clock64() - t0 > q.budget))
                break;
            __builtin_amdgcn_s_sleep(32);
        }
        if (e == 0) break;   // converged, or paused with this ticket unfilled
        const int g = (int)(uint32_t)e - 1;
        const int slot = (int)(e >> 32);
        if (lane == 0) {
            __hip_atomic_store(ep, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicExch(&q.state[g], 2);                      // being visited; clears "needs a visit"
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const MazeDev md = a.mazes[slot];
        const int lt = g - md.tile_base;
        const int ty = lt / md.tiles_x;
        const int tx = lt - ty * md.tiles_x;
        if (lane == 0) {
            const unsigned long long cells =
                (unsigned long long)tile_cells(md, ty, tx, a.tile_rows, a.tile_cols);
            const int sp = blockIdx.x & (kSpread - 1);
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_visits[slot * kSpread + sp]), 1ull);
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_cell_visits[slot * kSpread + sp]), cells);
            atomicAdd(a.total_cells + sp, cells);
            a.touched[g] = 1;
        }
        const bool changed = sweep_tile<T, C, true>(md, ty, tx, a.tile_rows, a.parity);
        // Every visit publishes its stores before it ends, changed or not: a
        // store left dirty in this XCD's L2 could otherwise be written back
        // after a later visit (on another XCD) stored larger values, and
        // overwrite them.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (changed) queue_mark_neighbourhood(q, md, slot, ty, tx);
        if (lane == 0) {
            const int old = atomicCAS(&q.state[g], 2, 0);
            if (old == 2) {
                if (atomicSub(q.pending, 1) == 1) __hip_atomic_store(q.done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                // marked while being visited: needs another visit (still pending)
                atomicExch(&q.state[g], 1);
                queue_push(q, g, slot);
            }
        }
    }
}

// After a paused launch: moves the entries still in the ring (in ring order)
// to a temporary array; the host copies them back to the ring's start and
// sets head = 0, tail = count.  One block.
__global__ __launch_bounds__(1024) void k_queue_gather(AsyncQueue q, unsigned long long* __restrict__ tmp,
                                                       uint32_t* __restrict__ count) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t base_s;
    if (threadIdx.x == 0) base_s = 0;
    __syncthreads();
    const uint32_t n = q.ring_mask + 1;
    for (uint32_t i0 = 0; i0 < n; i0 += 1024) {
        const uint32_t i = i0 + threadIdx.x;
        const unsigned long long e = i < n ? q.ring[i] : 0ull;
        const uint64_t m = __ballot(e != 0);
        const int w = threadIdx.x >> 6;
        if (lane_id() == 0) wsum[w] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = base_s;
        for (int k = 0; k < w; ++k) before += wsum[k];
        if (e != 0) {
            tmp[before + (uint32_t)__popcll(m & ((1ull << lane_id()) - 1))] = e;
            q.ring[i] = 0ull;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int k = 0; k < 16; ++k) base_s += wsum[k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base_s;
}

// One wave per tile of `slot`: zero the interior of touched tiles in both
// activity buffers (everything else is still 0 from the last full clear).
__global__ __launch_bounds__(kBlockThreads) void k_clear_touched(RoundArgs a, int32_t slot,
                                                                 int32_t n_tiles) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = blockIdx.x * kWavesPerBlock + wave;
    if (t >= n_tiles) return;
    const MazeDev md = a.mazes[slot];
    const int g = md.tile_base + t;
    if (!a.touched[g]) return;
    const int ty = t / md.tiles_x, tx = t - ty * md.tiles_x;
    const int r0 = ty * a.tile_rows, c0 = tx * a.tile_cols;
    const int rows = min(a.tile_rows, md.H - r0), cols = min(a.tile_cols, md.W - c0);
    for (int k = lane_id(); k < rows * cols; k += kLanes) {
        const int64_t x = (int64_t)(r0 + k / cols) * md.pitch + c0 + k % cols;
        md.V[0][x] = 0;
        md.V[1][x] = 0;
    }
    if (lane_id() == 0) a.touched[g] = 0;
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

__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ len, int32_t n,
                                               int64_t* __restrict__ off) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = min(n, t * chunk), e = min(n, b + chunk);
    int64_t s = 0;
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
    for (int i = b; i < e; ++i) {
        base += len[i] >= 0 ? (int64_t)len[i] + 1 : 0;
        off[i + 1] = base;
    }
}

__device__ __forceinline__ int dir_dr(int k) { return k < 3 ? -1 : (k < 5 ? 0 : 1); }
__device__ __forceinline__ int dir_dc(int k) {
    return (k == 0 || k == 3 || k == 5) ? -1 : ((k == 1 || k == 6) ? 0 : 1);
}

// The walk is a chain of dependent loads, one step after the other, so its
// time is the longest path times the latency of one step.  One wave follows
// one target: it loads a kWinRows x kWinCols window of the activity around the
// current cell into LDS with wide coalesced loads (one global round trip) and
// then takes up to kWinSteps steps from LDS, where a step costs a few LDS
// reads.  Window cells outside the grid read as -1, below every in-grid value.
constexpr int kWinRows = 32;
constexpr int kWinCols = 48;                   // 12 chunks of 4 columns
constexpr int kWinSteps = 15;                  // the window reaches >= 15 cells from its start in every direction
constexpr int kWinChunks = kWinRows * kWinCols / 4;
constexpr int kWalkWaves = 4;

__global__ __launch_bounds__(kLanes * kWalkWaves) void k_walk(
    const MazeDev* __restrict__ mazes, const int32_t* __restrict__ tslot, const int32_t* __restrict__ trc,
    int32_t n, int32_t parity, const int32_t* __restrict__ len, const int64_t* __restrict__ off,
    int32_t* __restrict__ cells) {
    __shared__ __attribute__((aligned(16))) int32_t win_all[kWalkWaves][kWinRows * kWinCols];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = lane_id();
    const int i = blockIdx.x * kWalkWaves + wave;
    if (i >= n) return;
    const int steps = __builtin_amdgcn_readfirstlane(len[i]);
    if (steps < 0) return;
    const int slot = __builtin_amdgcn_readfirstlane(tslot[i]);
    const MazeDev md = mazes[slot];
    const int32_t* __restrict__ V = parity ? md.V[1] : md.V[0];
    int32_t* win = win_all[wave];
    int r = __builtin_amdgcn_readfirstlane(trc[2 * i]);
    int c = __builtin_amdgcn_readfirstlane(trc[2 * i + 1]);
    int64_t o = off[i];
    if (lane == 0) cells[o] = r * md.W + c;
    ++o;
    for (int s = 0; s < steps;) {
        // window rows r-15 .. r+16, columns C0 .. C0+47 with C0 = 4*floor((c-16)/4)
        const int R0 = r - (kWinSteps), C0 = (c - 16) & ~3;
#pragma unroll
        for (int k = 0; k < kWinChunks / kLanes; ++k) {
            const int q = lane + kLanes * k;
            const int wr = q / (kWinCols / 4), wc = 4 * (q % (kWinCols / 4));
            const int R = R0 + wr, cs = C0 + wc;
            const bool rok = R >= 0 && R < md.H;
            const bool cok = cs >= 0 && cs < md.pitch;   // a chunk lies wholly inside or outside a row
            const v4i32 v = *(const __attribute__((address_space(1))) v4i32*)(
                V + (int64_t)(rok ? R : 0) * md.pitch + (cok ? cs : 0));
            v4i32 m;
#pragma unroll
            for (int e = 0; e < 4; ++e) m[e] = (rok && cs + e >= 0 && cs + e < md.W) ? v[e] : -1;
            *(__attribute__((address_space(3))) v4i32*)(win + wr * kWinCols + wc) = m;
        }
        // the same wave reads what its lanes wrote: LDS operations of a wave
        // complete in order; the wave barrier keeps the compiler from moving
        // the reads above the writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int lr = r - R0, lc = c - C0;
        const int todo = min(kWinSteps, steps - s);
        for (int k = 0; k < todo; ++k) {
            const int32_t* b = win + (lr - 1) * kWinCols + (lc - 1);
            const int nv[8] = {b[0], b[1], b[2], b[kWinCols], b[kWinCols + 2],
                               b[2 * kWinCols], b[2 * kWinCols + 1], b[2 * kWinCols + 2]};
            int best = 0, bv = nv[0];
#pragma unroll
            for (int j = 1; j < 8; ++j)
                if (nv[j] > bv) {
                    bv = nv[j];
                    best = j;
                }
            lr += dir_dr(best);
            lc += dir_dc(best);
            if (lane == 0) cells[o] = (R0 + lr) * md.W + (C0 + lc);
            ++o;
        }
        s += todo;
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
    const int64_t n4 = n_elems / 4;   // callers pass multiples of 4
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n4, 256, 65536)), dim3(256), 0, s, p, n4, value);
    return hipGetLastError();
}

hipError_t launch_check_sources(const uint32_t* mask, int32_t mpitch, const int32_t* src_rc,
                                int32_t n_src, int32_t* bad_count, hipStream_t s) {
    hipLaunchKernelGGL(k_check_sources, dim3(grid_for(n_src, 256)), dim3(256), 0, s, mask, mpitch,
                       src_rc, n_src, bad_count);
    return hipGetLastError();
}

hipError_t launch_seed(const RoundArgs& a, int32_t slot, const int32_t* src_rc, int32_t n_src,
                       int32_t* bad_count, hipStream_t s) {
    hipLaunchKernelGGL(k_seed, dim3(grid_for(n_src, 256)), dim3(256), 0, s, a, slot, src_rc, n_src,
                       a.dense ? 0 : 1, bad_count);
    return hipGetLastError();
}

hipError_t launch_slot_reset(const RoundArgs& a, int32_t slot, hipStream_t s) {
    hipLaunchKernelGGL(k_slot_reset, dim3(1), dim3(64), 0, s, a, slot);
    return hipGetLastError();
}

// Sweep kernels instantiated for (layers per visit, columns per lane).
#define OMAP_SWEEP_VARIANTS(X) \
    X(4, 4) X(8, 4) X(12, 4) X(16, 4) X(4, 2) X(8, 2) X(12, 2) X(16, 2) X(24, 2) X(32, 2)

hipError_t launch_sweep_persistent(int T, int C, const PersistentArgs& p, int32_t grid, hipStream_t s) {
    void* args[] = {const_cast<PersistentArgs*>(&p)};
#define X(t, c)                                                                                      \
    if (T == t && C == c)                                                                            \
        return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_sweep_persistent<t, c>),   \
                                          dim3(grid), dim3(kBlockThreads), args, 0, s);
    OMAP_SWEEP_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

int sweep_persistent_blocks_per_cu(int T, int C) {
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
#define X(t, c)                                                                                       \
    if (T == t && C == c)                                                                             \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep_persistent<t, c>, kBlockThreads, 0);
    OMAP_SWEEP_VARIANTS(X)
#undef X
    if (e != hipSuccess) blocks = 0;
    return blocks;
}

bool sweep_supported(int T, int C) {
#define X(t, c) if (T == t && C == c) return true;
    OMAP_SWEEP_VARIANTS(X)
#undef X
    return false;
}

hipError_t launch_sweep(int T, int C, const RoundArgs& a, int32_t grid, hipStream_t s) {
#define X(t, c)                                                                             \
    if (T == t && C == c) {                                                                 \
        hipLaunchKernelGGL((k_sweep<t, c>), dim3(grid), dim3(kBlockThreads), 0, s, a);     \
        return hipGetLastError();                                                           \
    }
    OMAP_SWEEP_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
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

hipError_t launch_scan_offsets(const int32_t* len, int32_t n, int64_t* offsets, hipStream_t s) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, len, n, offsets);
    return hipGetLastError();
}

hipError_t launch_walk(const MazeDev* mazes, const int32_t* tgt_slot, const int32_t* tgt_rc,
                       int32_t n_tgt, int32_t parity, const int32_t* len, const int64_t* offsets,
                       int32_t* cells, hipStream_t s) {
    if (n_tgt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk, dim3((n_tgt + kWalkWaves - 1) / kWalkWaves), dim3(kLanes * kWalkWaves), 0, s,
                       mazes, tgt_slot, tgt_rc, n_tgt, parity, len, offsets, cells);
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

hipError_t launch_clear_touched(const RoundArgs& a, int32_t slot, int32_t n_tiles, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_touched, dim3((n_tiles + kWavesPerBlock - 1) / kWavesPerBlock),
                       dim3(kBlockThreads), 0, s, a, slot, n_tiles);
    return hipGetLastError();
}

hipError_t launch_selftest(int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_selftest, dim3(1), dim3(64), 0, s, out);
    return hipGetLastError();
}

hipError_t launch_sweep_async(int T, int C, const RoundArgs& a, int32_t grid, hipStream_t s) {
#define X(t, c)                                                                                   \
    if (T == t && C == c) {                                                                       \
        hipLaunchKernelGGL((k_sweep_async<t, c>), dim3(grid), dim3(kBlockThreads), 0, s, a);     \
        return hipGetLastError();                                                                 \
    }
    OMAP_SWEEP_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_queue_compact(const AsyncQueue& q, unsigned long long* tmp, uint32_t* tmp_count, hipStream_t s) {
    hipLaunchKernelGGL(k_queue_gather, dim3(1), dim3(1024), 0, s, q, tmp, tmp_count);
    return hipGetLastError();
}

int sweep_async_waves_per_cu(int T, int C) {
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
#define X(t, c)                                                                                  \
    if (T == t && C == c)                                                                        \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep_async<t, c>, kBlockThreads, 0);
    OMAP_SWEEP_VARIANTS(X)
#undef X
    if (e != hipSuccess || blocks < 1) blocks = 1;
    return blocks * kWavesPerBlock;
}

int sweep_max_waves_per_cu(int T, int C) {
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
#define X(t, c)                                                                                  \
    if (T == t && C == c)                                                                        \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep<t, c>, kBlockThreads, 0);
    OMAP_SWEEP_VARIANTS(X)
#undef X
    if (e != hipSuccess || blocks < 1) blocks = 1;
    return blocks * kWavesPerBlock;
}

}  // namespace omap
