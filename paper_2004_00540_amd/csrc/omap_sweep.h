// Tile-sweep device code of the oMAP planner for gfx950 (CDNA4, wave64),
// compiled once per (layers per visit, columns per lane) variant by
// omap_sweep_variant.hip and included by omap_kernels.hip for the shared
// helpers (seeding uses the same scheduling functions).
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

#pragma once

#include "omap_internal.h"

#include <hip/hip_ext.h>

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
// Stages above SMAX (compile time) and, with GUARD, above smax (run time)
// are skipped (see sweep_tile).
template <int T, int P, int C, bool GUARD, int SMAX = T - 1>
__device__ __forceinline__ void sweep_row(uint32_t (&st)[T][3][C], uint32_t (&out)[C], int smax) {
    constexpr int PA = (P + 1) % 3, PB = (P + 2) % 3;
#pragma unroll
    for (int s = 0; s < T; ++s) {
        if (s <= SMAX && (!GUARD || s <= smax)) {
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
typedef int v1i32 __attribute__((ext_vector_type(1)));
template <int C> struct LaneVec;
template <> struct LaneVec<4> { typedef v4i32 type; };
template <> struct LaneVec<2> { typedef v2i32 type; };
template <> struct LaneVec<1> { typedef v1i32 type; };
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

// One row of the tile.  (v, w) holds row R, loaded D rows earlier; it is
// decoded into stage 0's slot P (cells outside the grid become exactly
// 0x80000000) and the same registers then receive the load of row R + D, whose
// latency overlaps the T-stage arithmetic of the next D rows.
// ROW is the row's step index in the visit when known at compile time
// (warm-up rows), -1 for a steady-state step (index >= 2T), -2 if unknown;
// bounds that follow from it are not tested at run time.
template <int T, int P, int C, bool GUARD, int D, int SMAX = T - 1, int ROW = -2>
__device__ __forceinline__ void sweep_iter(uint32_t (&st)[T][3][C], typename LaneVec<C>::type& v,
                                           uint32_t& w, const MazeDev& md,
                                           const int32_t* Vin, int32_t* Vout, int R, int r0, int r_end,
                                           int col, bool col_ok, bool inner, int smax,
                                           uint64_t& sum_in, uint64_t& sum_out) {
    constexpr bool kFromR0 = ROW == -1 || ROW >= T;          // R >= r0 (>= 0)
    constexpr bool kStoreFromR0 = ROW == -1 || ROW >= 2 * T;  // R - T >= r0
    constexpr bool kAboveTile = ROW >= 0 && ROW < T;          // R < r0
    constexpr bool kNotStored = ROW >= 0 && ROW < 2 * T;      // R - T < r0
    const bool ok = (kFromR0 || R >= 0) && R < md.H && col_ok;
    const uint32_t keep = ok ? 0xffffffffu : 0u;
    const uint32_t bits = ok ? (w >> (col & 31)) : 0xFu;   // outside the grid: obstacle
    uint32_t* c = st[0][P];
#pragma unroll
    for (int j = 0; j < C; ++j) c[j] = ((uint32_t)v[j] & keep) | (((bits >> j) & 1u) << 31);
    load_row<C>(md, Vin, R + D, col, col_ok, v, w);
    if (!kAboveTile && inner && (kFromR0 || R >= r0) && R < r_end) {
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) t += c[j] & 0x7fffffffu;
        sum_in += t;
    }
    uint32_t out[C] = {};   // left 0 when the last stage is skipped (its row is not stored then)
    sweep_row<T, P, C, GUARD, SMAX>(st, out, smax);
    const int Ro = R - T;
    if (!kNotStored && inner && (kStoreFromR0 || Ro >= r0) && Ro < r_end) {
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

// Rows of a tile visit whose loads are in flight at once.  A row's arithmetic
// (T stages) takes far less time than a load that misses the L2, so one group
// of three rows ahead leaves the wave waiting on memory; D rows ahead hide the
// latency.  A multiple of 3 (the pipeline's slot rotation).  Only the
// one-column variants prefetch 12 rows: their pipeline takes 3*T registers, and
// the wider variants, whose visits are longer anyway, compile to basic blocks
// that the instruction scheduler takes many minutes over when unrolled 4 times.
template <int T, int C>
struct SweepPrefetch {
    static constexpr int D = C == 1 ? 12 : 3;
};

// Rows R .. R + D - 1 of a visit: one sweep_iter per row with row buffer J
// and pipeline slot J mod 3 (compile-time indices, so everything stays in
// registers).  With GUARD, row R + J runs stages up to ((i + J) >> 1) - 1.
template <int T, int C, bool GUARD, int D, int J = 0>
__device__ __forceinline__ void sweep_rows(uint32_t (&st)[T][3][C], typename LaneVec<C>::type (&v)[D],
                                           uint32_t (&w)[D], const MazeDev& md, const int32_t* Vin,
                                           int32_t* Vout, int R, int i, int r0, int r_end, int col,
                                           bool col_ok, bool inner, uint64_t& sum_in, uint64_t& sum_out) {
    if constexpr (J < D) {
        sweep_iter<T, J % 3, C, GUARD, D, T - 1, GUARD ? -2 : -1>(st, v[J], w[J], md, Vin, Vout, R + J, r0, r_end,
                                                                  col, col_ok, inner,
                                                                  GUARD ? ((i + J) >> 1) - 1 : 0, sum_in, sum_out);
        sweep_rows<T, C, GUARD, D, J + 1>(st, v, w, md, Vin, Vout, R, i, r0, r_end, col, col_ok, inner, sum_in,
                                          sum_out);
    }
}

// The first KW rows of a visit (the top of the trapezoid, see sweep_tile)
// unrolled with each row's stage limit known at compile time: no run-time
// guards, and no code for the skipped stages.
template <int T, int C, int D, int KW, int I = 0>
__device__ __forceinline__ void sweep_warm(uint32_t (&st)[T][3][C], typename LaneVec<C>::type (&v)[D],
                                           uint32_t (&w)[D], const MazeDev& md, const int32_t* Vin,
                                           int32_t* Vout, int R0, int r0, int r_end, int col, bool col_ok,
                                           bool inner, uint64_t& sum_in, uint64_t& sum_out) {
    if constexpr (I < KW) {
        constexpr int SM = (I >> 1) - 1 < T - 1 ? (I >> 1) - 1 : T - 1;
        sweep_iter<T, I % 3, C, false, D, SM, I>(st, v[I % D], w[I % D], md, Vin, Vout, R0 + I, r0, r_end, col,
                                                 col_ok, inner, 0, sum_in, sum_out);
        sweep_warm<T, C, D, KW, I + 1>(st, v, w, md, Vin, Vout, R0, r0, r_end, col, col_ok, inner, sum_in,
                                       sum_out);
    }
}

// Returns true (wave-uniform) if any interior cell of the tile changed.  The
// wave streams the strip of 64*C columns starting T columns left of the tile.
template <int T, int C>
__device__ bool sweep_tile(const MazeDev& md, int ty, int tx, int tile_rows, int parity) {
    constexpr int TW = kLanes * C - 2 * T;
    constexpr int HALO_LANES = T / C;
    constexpr int D = SweepPrefetch<T, C>::D;
    const int lane = lane_id();
    const int r0 = ty * tile_rows;
    const int r_end = min(r0 + tile_rows, md.H);
    const int col = tx * TW - T + C * lane;
    const bool col_ok = col >= 0 && col < md.pitch;
    const bool inner = lane >= HALO_LANES && lane < kLanes - HALO_LANES && col < md.W;
    int32_t* const Vin = parity ? md.V[1] : md.V[0];
    int32_t* const Vout = parity ? md.V[0] : md.V[1];

    uint32_t st[T][3][C];
#pragma unroll
    for (int s = 0; s < T; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < C; ++j) st[s][k][j] = kObstacleBit;

    uint64_t sum_in = 0, sum_out = 0;
    const int n_iter = (r_end - r0) + 2 * T;   // rows r0-T .. r_end+T-1
    typename LaneVec<C>::type v[D];
    uint32_t w[D];
#pragma unroll
    for (int j = 0; j < D; ++j) load_row<C>(md, Vin, r0 - T + j, col, col_ok, v[j], w[j]);
    // Stage s at step i (input row r0 - T + i) emits row r0 - T + i - 1 - s
    // after s + 1 layers; the stored rows [r0, r_end) after T layers need
    // exactly the emissions with i >= 2s + 2 (each of which reads only
    // emissions of stage s - 1 with i - 2 >= 2(s - 1) + 2).  So during the
    // first 2T steps, stages s > i/2 - 1 are skipped: the top of the tile's
    // trapezoid, a third of the work of a tile with as many rows as layers.
    // Steps past n_iter (the last group's tail) store nothing.
    constexpr int kWarm = D * ((2 * T + D - 1) / D);   // >= 2T, a multiple of D
    int i = 0;
    if constexpr (C == 1) {
        // one column per lane: the warm-up unrolled (straight-line code of about
        // the size of one steady-state group for these depths)
        sweep_warm<T, C, D, kWarm>(st, v, w, md, Vin, Vout, r0 - T, r0, r_end, col, col_ok, inner, sum_in,
                                   sum_out);
        i = kWarm;
    } else {
#pragma unroll 1
        for (; i < kWarm; i += D)
            sweep_rows<T, C, true, D>(st, v, w, md, Vin, Vout, r0 - T + i, i, r0, r_end, col, col_ok, inner,
                                      sum_in, sum_out);
    }
#pragma unroll 1
    for (; i < n_iter; i += D)
        sweep_rows<T, C, false, D>(st, v, w, md, Vin, Vout, r0 - T + i, i, r0, r_end, col, col_ok, inner, sum_in,
                                   sum_out);
    return __ballot(sum_in != sum_out) != 0;
}

// Tile g of slot: T layers.  Returns true (wave-uniform) if the interior
// changed; md, ty, tx describe the tile.
template <int T, int C>
__device__ __forceinline__ bool visit_tile(const RoundArgs& a, int g, int slot, MazeDev& md, int& ty, int& tx) {
    md = a.n_slots == 1 ? a.md0 : a.mazes[slot];
    const int lt = g - md.tile_base;
    ty = lt / md.tiles_x;
    tx = lt - ty * md.tiles_x;
    return sweep_tile<T, C>(md, ty, tx, a.tile_rows, a.parity);
}

// Counters and flags of one visit (lane 0).  Called after the visit's own
// scheduling work: the vector-memory counter completes in issue order, so
// a load here issued before the tile's row loads would make the first row
// wait for these atomics and this load as well.
__device__ __forceinline__ void visit_bookkeeping(const RoundArgs& a, int g, int slot, const MazeDev& md,
                                                  int ty, int tx) {
    const unsigned long long cells = (unsigned long long)tile_cells(md, ty, tx, a.tile_rows, a.tile_cols);
    const int sp = blockIdx.x & (kSpread - 1);
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_visits[slot * kSpread + sp]), 1ull);
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_cell_visits[slot * kSpread + sp]), cells);
    atomicAdd(a.total_cells + sp, cells);
    a.touched[g] = 1;
    if (a.maze_last_round[slot] != a.round_id) a.maze_last_round[slot] = a.round_id;
}

// The same plus clearing the tile's scheduled flag of this round (active
// schedule), which lets the next round claim the tile again.
__device__ __forceinline__ void visit_bookkeeping_active(const RoundArgs& a, int g, int slot, const MazeDev& md,
                                                         int ty, int tx) {
    a.flags_in[g] = 0;
    visit_bookkeeping(a, g, slot, md, ty, tx);
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
    const int stride = a.wave_stride;
    int i = blockIdx.x * kWavesPerBlock + wave;
    // The first list entry is loaded before the count, so both round trips
    // overlap (the entry is in bounds for any i below the tile id space, and
    // used only if i < n).
    uint64_t e = 0;
    if (!a.dense && i < a.n_tile_ids) e = *reinterpret_cast<const uint64_t*>(a.list_in + 2 * i);
    const int n = a.dense ? a.n_tile_ids : __builtin_amdgcn_readfirstlane(*a.count_in);
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) *a.count_clear = 0;
        for (int m = threadIdx.x; m < a.n_slots; m += kBlockThreads) {
            a.sched_clear[m] = 0;
            a.dchg_clear[m] = 0;
        }
    }
    if (a.dense) {
        for (; i < n; i += stride) {
            const int slot = a.tile_maze[i];
            if (slot < 0 || __builtin_amdgcn_readfirstlane(a.dchg_prev[slot]) == 0) continue;
            MazeDev md;
            int ty, tx;
            const bool changed = visit_tile<T, C>(a, i, slot, md, ty, tx);
            if (lane == 0) {
                if (changed) {
                    a.dchg_cur[slot] = 1;
                    *a.count_out = 1;
                }
                visit_bookkeeping(a, i, slot, md, ty, tx);
            }
        }
        return;
    }
    // Active schedule.  The waves of a block take list entries ib .. ib+3
    // together, so that the tiles their changed tiles claim for the next
    // round are reserved with one atomic per block (same-address atomics
    // serialise device-wide).
    __shared__ int s_cnt[2][kWavesPerBlock];
    __shared__ int s_base[2];
    int par = 0;
    for (int ib = blockIdx.x * kWavesPerBlock; ib < n; ib += stride, par ^= 1) {
        i = ib + wave;
        int slot = 0, gn = 0, g = 0, ty = 0, tx = 0;
        bool won = false;
        MazeDev md;
        if (i < n) {
            g = __builtin_amdgcn_readfirstlane((int)(uint32_t)e);
            slot = __builtin_amdgcn_readfirstlane((int)(uint32_t)(e >> 32));
            if (i + stride < n) e = *reinterpret_cast<const uint64_t*>(a.list_in + 2 * (i + stride));
            if (visit_tile<T, C>(a, g, slot, md, ty, tx)) {
                // lanes 0..8 claim the 3x3 tiles around (ty, tx) for the next round
                const int ny = ty + lane / 3 - 1, nx = tx + lane % 3 - 1;
                gn = md.tile_base + ny * md.tiles_x + nx;
                if (lane < 9 && ny >= 0 && ny < md.tiles_y && nx >= 0 && nx < md.tiles_x)
                    won = atomicExch(&a.flags_out[gn], 1) == 0;
            }
        }
        const uint64_t wmask = __ballot(won);
        const int nwon = __popcll(wmask);
        if (lane == 0) s_cnt[par][wave] = nwon;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
#pragma unroll
            for (int w = 0; w < kWavesPerBlock; ++w) t += s_cnt[par][w];
            s_base[par] = t > 0 ? atomicAdd(a.count_out, t) : 0;
        }
        __syncthreads();
        if (nwon > 0) {
            int base = s_base[par];
            for (int w = 0; w < wave; ++w) base += s_cnt[par][w];
            if (won) {
                const int k = base + __popcll(wmask & ((1ull << lane) - 1));
                a.list_out[2 * k] = gn;
                a.list_out[2 * k + 1] = slot;
            }
            if (a.n_slots > 1 && lane == 0) atomicAdd(&a.sched_out[slot], nwon);
        }
        if (i < n && lane == 0) visit_bookkeeping_active(a, g, slot, md, ty, tx);
    }
}

template <int T, int C>
__global__ __launch_bounds__(kBlockThreads) void k_sweep(RoundArgs a) {
    if (a.round_base) a.round_id += *a.round_base;
    sweep_round<T, C>(a);
}

// Launch functions of one variant (defined in its own translation unit).
#define OMAP_DEFINE_SWEEP_VARIANT(t, c) OMAP_DEFINE_SWEEP_VARIANT_(t, c)
#define OMAP_DEFINE_SWEEP_VARIANT_(t, c)                                                              \
    hipError_t launch_sweep_T##t##_C##c(const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0, \
                                        hipEvent_t e1) {                                              \
        RoundArgs b = a;                                                                              \
        b.wave_stride = grid * kWavesPerBlock;                                                        \
        if (e0 != nullptr)                                                                            \
            hipExtLaunchKernelGGL((k_sweep<t, c>), dim3(grid), dim3(kBlockThreads), 0, s, e0, e1, 0, b); \
        else                                                                                          \
            hipLaunchKernelGGL((k_sweep<t, c>), dim3(grid), dim3(kBlockThreads), 0, s, b);           \
        return hipGetLastError();                                                                     \
    }                                                                                                 \
    int sweep_blocks_per_cu_T##t##_C##c() {                                                           \
        int blocks = 0;                                                                               \
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep<t, c>, kBlockThreads, 0); \
        return e == hipSuccess ? blocks : 0;                                                          \
    }

}  // namespace omap
