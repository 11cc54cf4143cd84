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

// Workgroup barrier for data exchanged through LDS only: the waves wait for
// their own LDS operations, not for their global stores and atomics, which
// __syncthreads also waits for (at the end of a visit that is the acknowledgement
// of the tile's output rows, about a microsecond).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// One stage of one row step: o = the layer applied to the centre row b with
// a and c above and below (C columns per lane).
template <int C>
__device__ __forceinline__ void sweep_stage(const uint32_t* a, const uint32_t* b, const uint32_t* c, uint32_t* o) {
    int v[C];
#pragma unroll
    for (int j = 0; j < C; ++j) v[j] = max3i((int)a[j], (int)b[j], (int)c[j]);
    const int left = from_left_lane(v[C - 1]);
    const int right = from_right_lane(v[0]);
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const int l = j == 0 ? left : v[j - 1];
        const int r = j == C - 1 ? right : v[j + 1];
        o[j] = max(b[j], sat_dec((uint32_t)max3i(l, v[j], r)));
    }
}

// Two independent stages computed operation by operation side by side (one
// column per lane), so that neither's DPP move waits on the instruction
// just before it.
__device__ __forceinline__ void sweep_stage_x2(const uint32_t* a0, const uint32_t* b0, const uint32_t* c0,
                                               uint32_t* o0, const uint32_t* a1, const uint32_t* b1,
                                               const uint32_t* c1, uint32_t* o1) {
    const int v0 = max3i((int)a0[0], (int)b0[0], (int)c0[0]);
    const int v1 = max3i((int)a1[0], (int)b1[0], (int)c1[0]);
    const int l0 = from_left_lane(v0);
    const int l1 = from_left_lane(v1);
    const int r0 = from_right_lane(v0);
    const int r1 = from_right_lane(v1);
    o0[0] = max(b0[0], sat_dec((uint32_t)max3i(l0, v0, r0)));
    o1[0] = max(b1[0], sat_dec((uint32_t)max3i(l1, v1, r1)));
}

// Two consecutive row steps (slots P and P + 1, stages up to SMAX in both)
// with their stage chains interleaved: stage s of the first step and stage
// s - 1 of the second use nothing the other computes, so each chain's
// instructions fill the other's DPP read-after-write gaps.  cnext is the
// second step's decoded input row; it enters stage 0's slot P + 1 once the
// first step's stage 0 has read the row it replaces.
template <int T, int P, int C, int SMAX>
__device__ __forceinline__ void sweep_row2(uint32_t (&st)[T][3][C], const uint32_t (&cnext)[C], uint32_t (&out0)[C],
                                           uint32_t (&out1)[C]) {
    constexpr int PA = (P + 1) % 3, PB = (P + 2) % 3;
#pragma unroll
    for (int s = 0; s <= T; ++s) {
        const bool first = s < T && s <= SMAX, second = s >= 1 && s - 1 <= SMAX;
        uint32_t* o0 = s + 1 < T ? st[s + 1 < T ? s + 1 : 0][P] : out0;
        uint32_t* o1 = s < T ? st[s < T ? s : 0][PA] : out1;
        if (C == 1 && first && second && s >= 1) {
            sweep_stage_x2(st[s][PA], st[s][PB], st[s][P], o0, st[s - 1][PB], st[s - 1][P], st[s - 1][PA], o1);
            continue;
        }
        if (first) sweep_stage<C>(st[s][PA], st[s][PB], st[s][P], o0);
        if (s == 0) {
#pragma unroll
            for (int j = 0; j < C; ++j) st[0][PA][j] = cnext[j];
        }
        if (second) sweep_stage<C>(st[s - 1][PB], st[s - 1][P], st[s - 1][PA], o1);
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

// Counters and flags of one visit of the dense schedule (lane 0).  Issued
// right after the visit's first D row loads: the vector-memory counter
// completes in issue order, so issued earlier they would delay the first row,
// and issued at the end of the visit their completion would delay the end of
// the kernel.  Issued here they complete while the first D rows are computed.
__device__ __forceinline__ void visit_bookkeeping(const RoundArgs& a, int g, int slot, const MazeDev& md,
                                                  int ty, int tx) {
    const unsigned long long cells = (unsigned long long)tile_cells(md, ty, tx, a.tile_rows, a.tile_cols);
    const int sp = blockIdx.x & (kSpread - 1);
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_visits[slot * kSpread + sp]), 1ull);
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_cell_visits[slot * kSpread + sp]), cells);
    atomicAdd(a.total_cells + sp, cells);
    a.touched[g] = 1;
    // every visiting wave of the round stores the same value (a test of the
    // old value first would make the wave wait for a load)
    a.maze_last_round[slot] = a.round_id;
}

// The same for a visit of a listed tile (active and bit-sliced schedules):
// the round's accounting block has counted the visit as one of full size
// (round_accounting), so only a tile cut by the maze's edge corrects the cell
// counts; and the tile's scheduled flag of this round is cleared, which lets
// the next round claim it again.
__device__ __forceinline__ void visit_bookkeeping_active(const RoundArgs& a, int g, int slot, const MazeDev& md,
                                                         int ty, int tx) {
    a.flags_in[g] = 0;
    a.touched[g] = 1;
    a.maze_last_round[slot] = a.round_id;
    const long long short_by = (long long)a.tile_rows * a.tile_cols - tile_cells(md, ty, tx, a.tile_rows, a.tile_cols);
    if (short_by != 0) {
        const int sp = blockIdx.x & (kSpread - 1);
        atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_cell_visits[slot * kSpread + sp]),
                  (unsigned long long)(-short_by));
        atomicAdd(a.total_cells + sp, (unsigned long long)(-short_by));
    }
}

// Work of the first block of a round launch, which visits no tile: it clears
// the buffers round r+2 will fill and (listed schedules) counts round r's
// visits from the list: per maze, its scheduled tiles (the whole list with
// one maze) as visits of full tiles, corrected by the visits of edge tiles.
// This replaces three same-address atomics per visit by one per maze and
// round, off the visiting waves' path.  BITS_T (bit-sliced schedule, its
// layers per visit): a maze whose rounds have covered its layers below K
// visits nothing.
template <int BITS_T, int NT = kBlockThreads>
__device__ __forceinline__ void round_accounting(const RoundArgs& a) {
    if (threadIdx.x == 0) *a.count_clear = 0;
    for (int m = threadIdx.x; m < a.n_slots; m += NT) {
        a.sched_clear[m] = 0;
        a.dchg_clear[m] = 0;
    }
    if (a.dense) return;
    const unsigned long long full = (unsigned long long)a.tile_rows * a.tile_cols;
    auto live = [&](const MazeDev& md) {
        return BITS_T == 0 || (int64_t)(a.round_id - md.round0) * BITS_T + 1 < md.K;
    };
    if (a.n_slots == 1) {
        if (threadIdx.x == 0) {
            const unsigned long long v = (unsigned long long)*a.count_in;
            if (v > 0 && live(a.md0)) {
                atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_visits[0]), v);
                atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_cell_visits[0]), v * full);
                atomicAdd(a.total_cells, v * full);
            }
        }
        return;
    }
    unsigned long long mine = 0;
    for (int m = threadIdx.x; m < a.n_slots; m += NT) {
        const unsigned long long v = (unsigned long long)a.sched_in[m];
        if (v > 0 && live(a.mazes[m])) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_visits[m * kSpread]), v);
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.maze_cell_visits[m * kSpread]), v * full);
            mine += v;
        }
    }
    for (int o = kLanes / 2; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
    if (lane_id() == 0 && mine > 0) atomicAdd(a.total_cells + (threadIdx.x >> 6), mine * full);
}

// ---- interior visits -------------------------------------------------------
//
// A visit whose rows all lie inside the maze (the T rows above the tile, the
// tile at its full height and every row prefetched below it) needs none of
// the row clamps, row validity tests and store bounds of the general visit.
// Its rows are addressed through buffer resources: a group of D row steps
// shares one base per buffer, and row step J of the group lies J row strides
// (a scalar offset) past it, so a row's loads and store cost no address
// arithmetic beyond the lane's column offset, computed once per visit.  The
// halo lanes' stores are dropped by the buffer range check (their offset is
// past the store resource's extent), so a row needs no branch around its
// store, and consecutive rows form one basic block that the compiler can
// interleave.  Row sums include the halo lanes; the final ballot ignores them.

// Lane constants of a visit.
struct VisitLane {
    int32_t voff;       // byte offset of the lane's first column in an activity row
    int32_t soff;       // the same for stores: voff for interior lanes, past the store extent for halo lanes
    int32_t moff;       // byte offset of the mask word holding the lane's columns
    int32_t vrow;       // activity row stride, bytes
    int32_t mrow;       // mask row stride, bytes
    uint32_t shift;     // bit of the lane's first column in its mask word
    bool col_ok, inner;
};

// Buffer resources of one group of D row steps starting at step i0: loads of
// the rows D steps ahead, and the stores of the rows T steps behind.
struct VisitGroup {
    __amdgpu_buffer_rsrc_t ldv, ldm, stv;
};

// Word 3 of a raw (untyped, unswizzled) buffer resource on this architecture
// family: 32-bit data format, everything else zero.
constexpr int kRawBufferWord3 = 0x00020000;
// Store offset of a halo lane: at or past any store resource's extent, so the
// range check drops the store (with or without the scalar offset added).
constexpr int32_t kDroppedStore = (int32_t)0x80000000u;

// Raw buffer resource over `bytes` bytes from base (accesses at offsets
// >= bytes are dropped: loads read 0, stores write nothing).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* base, int32_t bytes = 0x7fffffff) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, kRawBufferWord3);
}

template <int C>
__device__ __forceinline__ typename LaneVec<C>::type bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef typename LaneVec<C>::type V;
    if constexpr (C == 1) {
        V v;
        v[0] = (int)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        return v;
    } else if constexpr (C == 2) {
        return (V)__builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    } else {
        return (V)__builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    }
}

template <int C>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int voff, int soff, typename LaneVec<C>::type v) {
    if constexpr (C == 1) {
        __builtin_amdgcn_raw_buffer_store_b32((uint32_t)v[0], r, voff, soff, 0);
    } else if constexpr (C == 2) {
        typedef uint32_t U2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64((U2)v, r, voff, soff, 0);
    } else {
        typedef uint32_t U4 __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128((U4)v, r, voff, soff, 0);
    }
}

// Bases of the group starting at step i0 (row r0 - T + i0): loads go to row
// r0 - T + i0 + D + J, stores to row r0 - 2T + i0 + J.
// The store resource covers exactly the group's D output rows.
template <int T, int D>
__device__ __forceinline__ VisitGroup visit_group(const MazeDev& md, const int32_t* Vin, int32_t* Vout, int r0,
                                                  int i0) {
    VisitGroup g;
    g.ldv = raw_rsrc(Vin + (int64_t)(r0 - T + i0 + D) * md.pitch);
    g.ldm = raw_rsrc(md.mask + (int64_t)(r0 - T + i0 + D) * md.mpitch);
    g.stv = raw_rsrc(Vout + (int64_t)(r0 - 2 * T + i0) * md.pitch, D * md.pitch * 4);
    return g;
}

// Row step J of a group in an interior visit (sweep_iter without the row
// tests).  ROW is the step's index when known at compile time (warm-up), -1
// in the steady state, where `step` holds it.  Steps [T, sum_end) carry the
// tile's input rows, steps [2T, n_iter) emit its output rows.  In a steady
// group, SUM is false when no step of the group is below sum_end, and TAIL
// marks a last group that may run past n_iter.
template <int T, int P, int C, int J, int SMAX, int ROW, bool SUM = true, bool TAIL = false>
__device__ __forceinline__ void sweep_iter_inner(uint32_t (&st)[T][3][C], typename LaneVec<C>::type& v, uint32_t& w,
                                                 const VisitGroup& g, const VisitLane& L, int step, int sum_end,
                                                 int n_iter, uint64_t& sum_in, uint64_t& sum_out) {
    uint32_t* c = st[0][P];
    // missing columns (left of the maze, right of its pitch) decode as obstacles
#pragma unroll
    for (int j = 0; j < C; ++j) c[j] = L.col_ok ? (((w >> (L.shift + j)) << 31) | (uint32_t)v[j]) : kObstacleBit;
    v = bload<C>(g.ldv, L.voff, J * L.vrow);
    w = (uint32_t)bload<1>(g.ldm, L.moff, J * L.mrow)[0];
    constexpr bool kMaySum = SUM && (ROW < 0 || ROW >= T);
    if (kMaySum && (ROW < 0 ? step : ROW) < sum_end) {
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) t += c[j] & 0x7fffffffu;
        sum_in += t;
    }
    uint32_t out[C] = {};
    sweep_row<T, P, C, false, SMAX>(st, out, 0);
    constexpr bool kMayStore = ROW < 0 || ROW >= 2 * T;
    if (kMayStore && (!TAIL || step < n_iter)) {
        typename LaneVec<C>::type o;
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            o[j] = (int)(out[j] & 0x7fffffffu);
            t += (uint32_t)o[j];
        }
        bstore<C>(g.stv, L.soff, J * L.vrow, o);
        sum_out += t;
    }
}

// Row steps J and J + 1 of a group in an interior visit, their stages
// interleaved (sweep_row2); otherwise as two sweep_iter_inner steps.  Both
// steps share the stage limit SMAX (true for an even first warm-up step).
template <int T, int P, int C, int J, int SMAX, int ROW, bool SUM = true, bool TAIL = false>
__device__ __forceinline__ void sweep_iter2_inner(uint32_t (&st)[T][3][C], typename LaneVec<C>::type& v0,
                                                  uint32_t& w0, typename LaneVec<C>::type& v1, uint32_t& w1,
                                                  const VisitGroup& g, const VisitLane& L, int step, int sum_end,
                                                  int n_iter, uint64_t& sum_in, uint64_t& sum_out) {
    uint32_t* c0 = st[0][P];
    uint32_t c1[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
        c0[j] = L.col_ok ? (((w0 >> (L.shift + j)) << 31) | (uint32_t)v0[j]) : kObstacleBit;
        c1[j] = L.col_ok ? (((w1 >> (L.shift + j)) << 31) | (uint32_t)v1[j]) : kObstacleBit;
    }
    v0 = bload<C>(g.ldv, L.voff, J * L.vrow);
    w0 = (uint32_t)bload<1>(g.ldm, L.moff, J * L.mrow)[0];
    v1 = bload<C>(g.ldv, L.voff, (J + 1) * L.vrow);
    w1 = (uint32_t)bload<1>(g.ldm, L.moff, (J + 1) * L.mrow)[0];
    constexpr int ROW1 = ROW < 0 ? -1 : ROW + 1;
    constexpr bool kMaySum0 = SUM && (ROW < 0 || ROW >= T);
    constexpr bool kMaySum1 = SUM && (ROW1 < 0 || ROW1 >= T);
    if (kMaySum0 && (ROW < 0 ? step : ROW) < sum_end) {
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) t += c0[j] & 0x7fffffffu;
        sum_in += t;
    }
    if (kMaySum1 && (ROW1 < 0 ? step + 1 : ROW1) < sum_end) {
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) t += c1[j] & 0x7fffffffu;
        sum_in += t;
    }
    uint32_t out0[C] = {}, out1[C] = {};
    sweep_row2<T, P, C, SMAX>(st, c1, out0, out1);
    constexpr bool kMayStore0 = ROW < 0 || ROW >= 2 * T;
    constexpr bool kMayStore1 = ROW1 < 0 || ROW1 >= 2 * T;
    if (kMayStore0 && (!TAIL || step < n_iter)) {
        typename LaneVec<C>::type o;
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            o[j] = (int)(out0[j] & 0x7fffffffu);
            t += (uint32_t)o[j];
        }
        bstore<C>(g.stv, L.soff, J * L.vrow, o);
        sum_out += t;
    }
    if (kMayStore1 && (!TAIL || step + 1 < n_iter)) {
        typename LaneVec<C>::type o;
        uint64_t t = 0;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            o[j] = (int)(out1[j] & 0x7fffffffu);
            t += (uint32_t)o[j];
        }
        bstore<C>(g.stv, L.soff, (J + 1) * L.vrow, o);
        sum_out += t;
    }
}

// Steady-state group of an interior visit: steps i .. i + D - 1 (SUM: some
// of them below sum_end; TAIL: the last group, which may run past n_iter).
template <int T, int C, int D, bool SUM, bool TAIL, int J = 0>
__device__ __forceinline__ void sweep_rows_inner(uint32_t (&st)[T][3][C], typename LaneVec<C>::type (&v)[D],
                                                 uint32_t (&w)[D], const VisitGroup& g, const VisitLane& L, int i,
                                                 int sum_end, int n_iter, uint64_t& sum_in, uint64_t& sum_out) {
    if constexpr (J + 1 < D) {
        sweep_iter2_inner<T, J % 3, C, J, T - 1, -1, SUM, TAIL>(st, v[J], w[J], v[J + 1], w[J + 1], g, L, i + J,
                                                                sum_end, n_iter, sum_in, sum_out);
        sweep_rows_inner<T, C, D, SUM, TAIL, J + 2>(st, v, w, g, L, i, sum_end, n_iter, sum_in, sum_out);
    } else if constexpr (J < D) {
        sweep_iter_inner<T, J % 3, C, J, T - 1, -1, SUM, TAIL>(st, v[J], w[J], g, L, i + J, sum_end, n_iter,
                                                               sum_in, sum_out);
    }
}

// Warm-up of an interior visit: steps 0 .. KW - 1 unrolled, stage limits and
// store steps known at compile time (KW <= n_iter, so every warm-up step at
// or past 2T stores).
template <int T, int C, int D, int KW, int I = 0>
__device__ __forceinline__ void sweep_warm_inner(uint32_t (&st)[T][3][C], typename LaneVec<C>::type (&v)[D],
                                                 uint32_t (&w)[D], VisitGroup& g, const MazeDev& md,
                                                 const int32_t* Vin, int32_t* Vout, int r0, const VisitLane& L,
                                                 int sum_end, int n_iter, uint64_t& sum_in, uint64_t& sum_out) {
    if constexpr (I + 1 < KW && I % 2 == 0 && (I + 1) % D != 0) {
        // steps I and I + 1 (I even: same stage limit) in one group
        constexpr int SM = (I >> 1) - 1 < T - 1 ? (I >> 1) - 1 : T - 1;
        if constexpr (I % D == 0) g = visit_group<T, D>(md, Vin, Vout, r0, I);
        sweep_iter2_inner<T, I % 3, C, I % D, SM, I>(st, v[I % D], w[I % D], v[(I + 1) % D], w[(I + 1) % D], g, L,
                                                     I, sum_end, n_iter, sum_in, sum_out);
        sweep_warm_inner<T, C, D, KW, I + 2>(st, v, w, g, md, Vin, Vout, r0, L, sum_end, n_iter, sum_in, sum_out);
    } else if constexpr (I < KW) {
        constexpr int SM = (I >> 1) - 1 < T - 1 ? (I >> 1) - 1 : T - 1;
        if constexpr (I % D == 0) g = visit_group<T, D>(md, Vin, Vout, r0, I);
        sweep_iter_inner<T, I % 3, C, I % D, SM, I>(st, v[I % D], w[I % D], g, L, I, sum_end, n_iter, sum_in,
                                                    sum_out);
        sweep_warm_inner<T, C, D, KW, I + 1>(st, v, w, g, md, Vin, Vout, r0, L, sum_end, n_iter, sum_in, sum_out);
    }
}

// An interior visit (see above); same result as the general one.  on_start()
// runs once the first D rows' loads are issued.
template <int T, int C, class OnStart>
__device__ __forceinline__ bool sweep_tile_inner(const MazeDev& md, int r0, int tile_rows, const VisitLane& L,
                                                 const int32_t* Vin, int32_t* Vout, OnStart& on_start) {
    constexpr int D = SweepPrefetch<T, C>::D;
    constexpr int kWarm = D * ((2 * T + D - 1) / D);
    uint32_t st[T][3][C];
#pragma unroll
    for (int s = 0; s < T; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < C; ++j) st[s][k][j] = kObstacleBit;
    uint64_t sum_in = 0, sum_out = 0;
    const int n_iter = tile_rows + 2 * T;
    const int sum_end = T + tile_rows;
    typename LaneVec<C>::type v[D];
    uint32_t w[D];
    {
        const __amdgpu_buffer_rsrc_t rv = raw_rsrc(Vin + (int64_t)(r0 - T) * md.pitch);
        const __amdgpu_buffer_rsrc_t rm = raw_rsrc(md.mask + (int64_t)(r0 - T) * md.mpitch);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            v[j] = bload<C>(rv, L.voff, j * L.vrow);
            w[j] = (uint32_t)bload<1>(rm, L.moff, j * L.mrow)[0];
        }
    }
    on_start();
    VisitGroup g;
    sweep_warm_inner<T, C, D, kWarm>(st, v, w, g, md, Vin, Vout, r0, L, sum_end, n_iter, sum_in, sum_out);
    int i = kWarm;
#pragma unroll 1
    for (; i + D <= n_iter; i += D) {
        g = visit_group<T, D>(md, Vin, Vout, r0, i);
        if (i < sum_end)
            sweep_rows_inner<T, C, D, true, false>(st, v, w, g, L, i, sum_end, n_iter, sum_in, sum_out);
        else
            sweep_rows_inner<T, C, D, false, false>(st, v, w, g, L, i, sum_end, n_iter, sum_in, sum_out);
    }
    if (i < n_iter) {
        g = visit_group<T, D>(md, Vin, Vout, r0, i);
        sweep_rows_inner<T, C, D, true, true>(st, v, w, g, L, i, sum_end, n_iter, sum_in, sum_out);
    }
    return __ballot(L.inner && sum_in != sum_out) != 0;
}

// Returns true (wave-uniform) if any interior cell of the tile changed.  The
// wave streams the strip of 64*C columns starting T columns left of the tile.
// on_start() runs once the loads of the visit's first D rows are issued.
template <int T, int C, class OnStart>
__device__ bool sweep_tile(const MazeDev& md, int ty, int tx, int tile_rows, int parity, OnStart& on_start) {
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
    if constexpr (C == 1) {
        // interior visit: every loaded row inside the maze (the last group of
        // D steps may run past n_iter and prefetch D rows beyond it), full
        // tile height, and a warm-up that ends inside the visit
        constexpr int kWarmI = D * ((2 * T + D - 1) / D);
        if (r0 >= T && r_end == r0 + tile_rows && tile_rows + 2 * T >= kWarmI &&
            (int64_t)r0 + tile_rows + T + 2 * D <= md.H) {
            VisitLane L;
            const int cc = col_ok ? col : 0;
            L.voff = cc * 4;
            L.soff = inner ? L.voff : kDroppedStore;
            L.moff = (cc >> 5) * 4;
            L.vrow = md.pitch * 4;
            L.mrow = md.mpitch * 4;
            L.shift = (uint32_t)(col & 31);
            L.col_ok = col_ok;
            L.inner = inner;
            return sweep_tile_inner<T, C>(md, r0, tile_rows, L, Vin, Vout, on_start);
        }
    }

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
    on_start();
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

// Tile g of slot: T layers, with the visit's bookkeeping (ACTIVE: also the
// tile's scheduled flag).  Returns true (wave-uniform) if the interior
// changed; md, ty, tx describe the tile.
template <int T, int C, bool ACTIVE>
__device__ __forceinline__ bool visit_tile(const RoundArgs& a, int g, int slot, MazeDev& md, int& ty, int& tx) {
    md = a.n_slots == 1 ? a.md0 : a.mazes[slot];
    const int lt = g - md.tile_base;
    ty = lt / md.tiles_x;
    tx = lt - ty * md.tiles_x;
    const MazeDev& m = md;
    const int y = ty, x = tx;
    auto on_start = [&]() {
        if (lane_id() == 0) {
            if (ACTIVE)
                visit_bookkeeping_active(a, g, slot, m, y, x);
            else
                visit_bookkeeping(a, g, slot, m, y, x);
        }
    };
    return sweep_tile<T, C>(md, ty, tx, a.tile_rows, a.parity, on_start);
}

// Round r: every scheduled tile gets T layers.  Active schedule: the tiles of
// a.list_in; a changed tile schedules itself and its 8 neighbour tiles for
// round r+1.  Dense schedule: every tile of each maze that changed in round
// r-1; a changed tile flags its maze for round r+1.  Block 0 also clears the
// buffers round r+1 will fill.
// e0 (this wave's first list entry) and cnt (the round's count) were loaded
// by the kernel before anything else (see k_sweep).
template <int T, int C>
__device__ __forceinline__ void sweep_round(const RoundArgs& a, uint64_t e0, int cnt) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = lane_id();
    const int stride = a.wave_stride;
    int i = (blockIdx.x - 1) * kWavesPerBlock + wave;   // block 0: the accounting block
    uint64_t e = e0;
    const int n = a.dense ? a.n_tile_ids : __builtin_amdgcn_readfirstlane(cnt);
    if (a.dense) {
        for (; i < n; i += stride) {
            const int slot = a.tile_maze[i];
            if (slot < 0 || __builtin_amdgcn_readfirstlane(a.dchg_prev[slot]) == 0) continue;
            MazeDev md;
            int ty, tx;
            const bool changed = visit_tile<T, C, false>(a, i, slot, md, ty, tx);
            if (lane == 0 && changed) {
                a.dchg_cur[slot] = 1;
                *a.count_out = 1;
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
    for (int ib = (blockIdx.x - 1) * kWavesPerBlock; ib < n; ib += stride, par ^= 1) {
        i = ib + wave;
        int slot = 0, gn = 0, g = 0, ty = 0, tx = 0;
        bool won = false;
        MazeDev md;
        if (i < n) {
            g = __builtin_amdgcn_readfirstlane((int)(uint32_t)e);
            slot = __builtin_amdgcn_readfirstlane((int)(uint32_t)(e >> 32));
            if (i + stride < n) e = *reinterpret_cast<const uint64_t*>(a.list_in + 2 * (i + stride));
            if (visit_tile<T, C, true>(a, g, slot, md, ty, tx)) {
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
        lds_barrier();
        if (threadIdx.x == 0) {
            int t = 0;
#pragma unroll
            for (int w = 0; w < kWavesPerBlock; ++w) t += s_cnt[par][w];
            s_base[par] = t > 0 ? atomicAdd(a.count_out, t) : 0;
        }
        lds_barrier();
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
    }
}

// The grid has one block more than a.wave_stride covers: the first one (the
// first dispatched) does the round's accounting (round_accounting) instead
// of visits.
template <int T, int C>
__global__ __launch_bounds__(kBlockThreads) void k_sweep(RoundArgs a) {
    // This wave's first list entry and the round's count start the round's
    // longest chain of dependent loads: they are issued before anything else,
    // together, with no branch between them (the entry's index is clamped
    // into the list and the entry used only if it is below the count; relaxed
    // atomic loads of workgroup scope are plain cached loads that the
    // compiler keeps where they are written; the previous round's writes are
    // visible across the kernel boundary).
    const int i = ((int)blockIdx.x - 1) * kWavesPerBlock + (int)(threadIdx.x >> 6);
    const int ie = i >= 0 && i < a.n_tile_ids ? i : 0;
    const uint64_t e0 = __hip_atomic_load(reinterpret_cast<const uint64_t*>(a.list_in + 2 * ie), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
    const int cnt = __hip_atomic_load(a.count_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (a.round_base) a.round_id += *a.round_base;
    if (blockIdx.x == 0) {
        round_accounting<0>(a);
        return;
    }
    sweep_round<T, C>(a, e0, cnt);
}

// Launch functions of one variant (defined in its own translation unit).
#define OMAP_DEFINE_SWEEP_VARIANT(t, c) OMAP_DEFINE_SWEEP_VARIANT_(t, c)
#define OMAP_DEFINE_SWEEP_VARIANT_(t, c)                                                              \
    hipError_t launch_sweep_T##t##_C##c(const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0, \
                                        hipEvent_t e1) {                                              \
        RoundArgs b = a;                                                                              \
        b.wave_stride = grid * kWavesPerBlock;                                                        \
        if (e0 != nullptr)                                                                            \
            hipExtLaunchKernelGGL((k_sweep<t, c>), dim3(grid + 1), dim3(kBlockThreads), 0, s, e0, e1, 0, b); \
        else                                                                                          \
            hipLaunchKernelGGL((k_sweep<t, c>), dim3(grid + 1), dim3(kBlockThreads), 0, s, b);       \
        return hipGetLastError();                                                                     \
    }                                                                                                 \
    int sweep_blocks_per_cu_T##t##_C##c() {                                                           \
        int blocks = 0;                                                                               \
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep<t, c>, kBlockThreads, 0); \
        return e == hipSuccess ? blocks : 0;                                                          \
    }

}  // namespace omap
