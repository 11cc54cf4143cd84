// Two-wave tile visits: the T stages of a one-column-per-lane visit split
// between the waves of a workgroup (two; three also build).
//
// A round of the active schedule on a single large maze has a few hundred
// tiles for 1024 SIMDs, so its time is one visit's latency, and a visit is a
// chain of T stages over TH + 2T row steps issued by one wave.  Here wave A
// loads the rows and runs stages 0 .. S1-1, wave B runs stages S1 .. T-1 and
// stores the rows: A hands each row that its last stage emits to B through
// an LDS ring (one slot per row step, so it never wraps) and publishes how
// many it has written; B waits only when it has caught up.  The split point
// S1 = 3T/8 balances the two waves' stage-rows (the trapezoid's top, where
// the first stages already run and the last do not, is all A's).  The
// result is bit-identical to the one-wave visit: every stage sees the same
// rows in the same order; only the wave that computes it differs.
//
// Tiles of TH = T rows (every row step's stage limit is then a compile-time
// constant).  Wave A addresses an interior tile's rows through buffer
// resources (the interior visits of omap_sweep.h) and clamps the rows of a
// tile near the maze's top or bottom edge, where rows outside the maze
// decode as obstacles; wave B drops the rows of a tile cut by the bottom
// edge (store range and output sums).
#pragma once

#include "omap_sweep.h"

// Waves per visit: 2 (three, with stages 0-3, 4-8 and 9-15, measured slower
// on the 23170^2 maze: 6.48 vs 6.35 ms per propagation, as a 25 KB LDS ring
// pair per tile leaves room for 1536 tiles in flight against 2048).
#ifndef OMAP_SPLIT_WAVES
#define OMAP_SPLIT_WAVES 2
#endif

namespace omap {

// Waves per tile visit and the first stage of each wave (stage-rows balanced
// over the trapezoid: the first stages have the most rows).
constexpr int kSplitWaves = OMAP_SPLIT_WAVES;
constexpr int kSplitThreads = kSplitWaves * kLanes;

template <int T>
struct SplitVisit {
    static constexpr int NW = kSplitWaves;
    static constexpr int first_stage(int k) {
        return NW == 2 ? (k == 0 ? 0 : (k == 1 ? 3 * T / 8 : T))
                       : (k == 0 ? 0 : (k == 1 ? T / 4 : (k == 2 ? 9 * T / 16 : T)));
    }
    static constexpr int S1 = first_stage(1);     // stages of wave A
    static constexpr int NSTEP = 3 * T;           // row steps of a tile with TH = T
    static constexpr int D = SweepPrefetch<T, 1>::D;
    static_assert(NW == 2 || NW == 3, "two or three waves per visit");
    static_assert(NSTEP % 2 == 0 && D % 6 == 0, "split visit steps");
};

// LDS of one split visit: ring k carries the rows emitted by the last stage
// of wave k to wave k + 1.
template <int T>
struct SplitShared {
    int32_t ring[kSplitWaves - 1][SplitVisit<T>::NSTEP][kLanes];
    uint64_t sum_in[kLanes];                      // wave A's input sums
    int32_t ready[kSplitWaves - 1];               // rows written to ring k (a count of steps)
    int32_t done;                                 // 1 once sum_in is written
};

__device__ __forceinline__ void lds_publish(int32_t* p, int32_t v) {
    if (lane_id() == 0) __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Waits until *p >= need (wave-uniform); `seen` caches the last value read.
// The waves of a workgroup run (and are suspended) together and wave A never
// waits on a later wave, so the wait ends within a visit (microseconds); the
// spin bound (about 30 ms) only keeps a broken invariant from hanging the GPU.
__device__ __forceinline__ void lds_wait_at_least(const int32_t* p, int32_t need, int32_t& seen) {
    for (int spin = 0; seen < need && spin < (1 << 20); ++spin) {
        seen = __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (seen < need) __builtin_amdgcn_s_sleep(1);
    }
}

// Wave A, row steps I and I + 1 (I even, compile time): decode, prefetch,
// input sums, stages 0 .. S1-1 (limited by the trapezoid), hand the emitted
// rows to wave B.  EDGE: rows clamped into the maze (row r0 - T + I of the
// visit is row R0 + I of the maze), rows outside it obstacles, and only the
// rows below r_end summed.
template <int T, int I, bool EDGE>
__device__ __forceinline__ void split_a_pair(uint32_t (&st)[SplitVisit<T>::S1][3][1], v1i32 (&v)[SplitVisit<T>::D],
                                             uint32_t (&w)[SplitVisit<T>::D], VisitGroup& g, const MazeDev& md,
                                             const int32_t* Vin, int r0, int r_end, int col, const VisitLane& L,
                                             uint64_t& sum_in, SplitShared<T>& sh) {
    using SV = SplitVisit<T>;
    constexpr int D = SV::D, S1 = SV::S1;
    constexpr int J = I % D;
    constexpr int P = I % 3;
    constexpr int SM = (I >> 1) - 1 < S1 - 1 ? (I >> 1) - 1 : S1 - 1;
    uint32_t c1[1];
    if constexpr (EDGE) {
        const int R = r0 - T + I;
        const bool ok0 = R >= 0 && R < md.H && L.col_ok, ok1 = R + 1 >= 0 && R + 1 < md.H && L.col_ok;
        st[0][P][0] = ok0 ? (((w[J] >> L.shift) << 31) | (uint32_t)v[J][0]) : kObstacleBit;
        c1[0] = ok1 ? (((w[J + 1] >> L.shift) << 31) | (uint32_t)v[J + 1][0]) : kObstacleBit;
        load_row<1>(md, Vin, R + D, col, L.col_ok, v[J], w[J]);
        load_row<1>(md, Vin, R + 1 + D, col, L.col_ok, v[J + 1], w[J + 1]);
        if constexpr (I >= T && I < 2 * T)
            if (R < r_end) sum_in += st[0][P][0] & 0x7fffffffu;
        if constexpr (I + 1 >= T && I + 1 < 2 * T)
            if (R + 1 < r_end) sum_in += c1[0] & 0x7fffffffu;
    } else {
        if constexpr (J == 0) g = visit_group<T, D>(md, Vin, const_cast<int32_t*>(Vin), r0, I);   // (A stores nothing)
        st[0][P][0] = L.col_ok ? (((w[J] >> L.shift) << 31) | (uint32_t)v[J][0]) : kObstacleBit;
        c1[0] = L.col_ok ? (((w[J + 1] >> L.shift) << 31) | (uint32_t)v[J + 1][0]) : kObstacleBit;
        v[J] = bload<1>(g.ldv, L.voff, J * L.vrow);
        w[J] = (uint32_t)bload<1>(g.ldm, L.moff, J * L.mrow)[0];
        v[J + 1] = bload<1>(g.ldv, L.voff, (J + 1) * L.vrow);
        w[J + 1] = (uint32_t)bload<1>(g.ldm, L.moff, (J + 1) * L.mrow)[0];
        // the tile's input rows are steps T .. 2T-1 (TH = T)
        if constexpr (I >= T && I < 2 * T) sum_in += st[0][P][0] & 0x7fffffffu;
        if constexpr (I + 1 >= T && I + 1 < 2 * T) sum_in += c1[0] & 0x7fffffffu;
    }
    uint32_t out0[1] = {}, out1[1] = {};
    sweep_row2<S1, P, 1, SM>(st, c1, out0, out1);
    if constexpr (I + 1 >= 2 * S1) {
        if constexpr (I >= 2 * S1) sh.ring[0][I][lane_id()] = (int32_t)out0[0];
        sh.ring[0][I + 1][lane_id()] = (int32_t)out1[0];
        lds_publish(&sh.ready[0], I + 2);
    }
}

template <int T, bool EDGE, int I = 0>
__device__ __forceinline__ void split_a_steps(uint32_t (&st)[SplitVisit<T>::S1][3][1], v1i32 (&v)[SplitVisit<T>::D],
                                              uint32_t (&w)[SplitVisit<T>::D], VisitGroup& g, const MazeDev& md,
                                              const int32_t* Vin, int r0, int r_end, int col, const VisitLane& L,
                                              uint64_t& sum_in, SplitShared<T>& sh) {
    if constexpr (I < SplitVisit<T>::NSTEP) {
        split_a_pair<T, I, EDGE>(st, v, w, g, md, Vin, r0, r_end, col, L, sum_in, sh);
        split_a_steps<T, EDGE, I + 2>(st, v, w, g, md, Vin, r0, r_end, col, L, sum_in, sh);
    }
}

// Wave A's part of a visit.
template <int T, bool EDGE, class OnStart>
__device__ __forceinline__ void split_wave_a(const MazeDev& md, int r0, int r_end, int col, const VisitLane& L,
                                             const int32_t* Vin, SplitShared<T>& sh, OnStart& on_start) {
    using SV = SplitVisit<T>;
    uint32_t st[SV::S1][3][1];
#pragma unroll
    for (int s = 0; s < SV::S1; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) st[s][k][0] = kObstacleBit;
    v1i32 v[SV::D];
    uint32_t w[SV::D];
    if constexpr (EDGE) {
#pragma unroll
        for (int j = 0; j < SV::D; ++j) load_row<1>(md, Vin, r0 - T + j, col, L.col_ok, v[j], w[j]);
    } else {
        const __amdgpu_buffer_rsrc_t rv = raw_rsrc(Vin + (int64_t)(r0 - T) * md.pitch);
        const __amdgpu_buffer_rsrc_t rm = raw_rsrc(md.mask + (int64_t)(r0 - T) * md.mpitch);
#pragma unroll
        for (int j = 0; j < SV::D; ++j) {
            v[j] = bload<1>(rv, L.voff, j * L.vrow);
            w[j] = (uint32_t)bload<1>(rm, L.moff, j * L.mrow)[0];
        }
    }
    on_start();
    uint64_t sum_in = 0;
    VisitGroup g;
    split_a_steps<T, EDGE>(st, v, w, g, md, Vin, r0, r_end, col, L, sum_in, sh);
    sh.sum_in[lane_id()] = sum_in;
    lds_publish(&sh.done, 1);
}

// Wave K >= 1, row steps I and I + 1: stages first_stage(K) .. first_stage(K
// + 1) - 1 on the rows the previous wave handed over (read one pair ahead);
// the last wave stores the tile's output rows, the others hand their rows on.
template <int T, int K, int I>
__device__ __forceinline__ void split_c_pair(
    uint32_t (&st)[SplitVisit<T>::first_stage(K + 1) - SplitVisit<T>::first_stage(K)][3][1], int32_t (&nxt)[2],
    __amdgpu_buffer_rsrc_t stv, const VisitLane& L, int rows, uint64_t& sum_out, SplitShared<T>& sh,
    int32_t& seen) {
    using SV = SplitVisit<T>;
    constexpr int B0 = SV::first_stage(K), B1 = SV::first_stage(K + 1), S = B1 - B0;
    constexpr bool LAST = K == SV::NW - 1;
    constexpr int P = I % 3;
    constexpr int SMG = (I >> 1) - 1 - B0;     // last active stage of this wave (local index), if >= 0
    constexpr int SM = SMG < S - 1 ? SMG : S - 1;
    st[0][P][0] = (uint32_t)nxt[0];
    uint32_t c1[1] = {(uint32_t)nxt[1]};
    if constexpr (I + 2 < SV::NSTEP) {
        lds_wait_at_least(&sh.ready[K - 1], I + 4, seen);
        nxt[0] = sh.ring[K - 1][I + 2][lane_id()];
        nxt[1] = sh.ring[K - 1][I + 3][lane_id()];
    }
    uint32_t out0[1] = {}, out1[1] = {};
    sweep_row2<S, P, 1, SM>(st, c1, out0, out1);
    if constexpr (LAST && I >= 2 * T) {
        // rows at or past the tile's `rows` (a tile cut by the maze's bottom
        // edge) lie outside the store resource and are left out of the sums
        // (the row offset is in the lane offset, which the range check covers)
        const uint32_t o0 = out0[0] & 0x7fffffffu, o1 = out1[0] & 0x7fffffffu;
        bstore<1>(stv, L.soff + (I - 2 * T) * L.vrow, 0, v1i32{(int)o0});
        bstore<1>(stv, L.soff + (I + 1 - 2 * T) * L.vrow, 0, v1i32{(int)o1});
        sum_out += (I - 2 * T < rows ? (uint64_t)o0 : 0) + (I + 1 - 2 * T < rows ? (uint64_t)o1 : 0);
    }
    if constexpr (!LAST && I + 1 >= 2 * B1) {
        if constexpr (I >= 2 * B1) sh.ring[K][I][lane_id()] = (int32_t)out0[0];
        sh.ring[K][I + 1][lane_id()] = (int32_t)out1[0];
        lds_publish(&sh.ready[K], I + 2);
    }
}

template <int T, int K, int I = 2 * SplitVisit<T>::first_stage(K)>
__device__ __forceinline__ void split_c_steps(
    uint32_t (&st)[SplitVisit<T>::first_stage(K + 1) - SplitVisit<T>::first_stage(K)][3][1], int32_t (&nxt)[2],
    __amdgpu_buffer_rsrc_t stv, const VisitLane& L, int rows, uint64_t& sum_out, SplitShared<T>& sh,
    int32_t& seen) {
    if constexpr (I < SplitVisit<T>::NSTEP) {
        split_c_pair<T, K, I>(st, nxt, stv, L, rows, sum_out, sh, seen);
        split_c_steps<T, K, I + 2>(st, nxt, stv, L, rows, sum_out, sh, seen);
    }
}

// Wave K >= 1's part of a visit; the last wave returns (wave-uniform) whether
// the interior changed.
template <int T, int K>
__device__ __forceinline__ bool split_wave_c(const MazeDev& md, int r0, const VisitLane& L, int32_t* Vout,
                                             SplitShared<T>& sh) {
    using SV = SplitVisit<T>;
    constexpr int B0 = SV::first_stage(K), S = SV::first_stage(K + 1) - B0;
    uint32_t st[S][3][1];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) st[s][k][0] = kObstacleBit;
    const int rows = min(r0 + T, md.H) - r0;
    const __amdgpu_buffer_rsrc_t stv = raw_rsrc(Vout + (int64_t)r0 * md.pitch, rows * md.pitch * 4);
    int32_t seen = 0;
    int32_t nxt[2];
    lds_wait_at_least(&sh.ready[K - 1], 2 * B0 + 2, seen);
    nxt[0] = sh.ring[K - 1][2 * B0][lane_id()];
    nxt[1] = sh.ring[K - 1][2 * B0 + 1][lane_id()];
    uint64_t sum_out = 0;
    split_c_steps<T, K>(st, nxt, stv, L, rows, sum_out, sh, seen);
    if constexpr (K == SV::NW - 1) {
        int32_t fin = 0;
        lds_wait_at_least(&sh.done, 1, fin);
        const uint64_t sum_in = sh.sum_in[lane_id()];
        return __ballot(L.inner && sum_in != sum_out) != 0;
    }
    return false;
}

// The visit of a tile with TH = T by the workgroup's waves (wave 0 = A);
// returns (wave-uniform, in the last wave) whether the interior changed.
// on_start() runs in wave A once its first D rows' loads are issued.
template <int T, class OnStart>
__device__ __forceinline__ bool split_visit(int wave, const MazeDev& md, int r0, int col, const VisitLane& L,
                                            const int32_t* Vin, int32_t* Vout, SplitShared<T>& sh,
                                            OnStart& on_start) {
    using SV = SplitVisit<T>;
    if (wave == 0) {
        const int r_end = min(r0 + T, md.H);
        if (r0 >= T && (int64_t)r0 + T + T + 2 * SV::D <= md.H)
            split_wave_a<T, false>(md, r0, r_end, col, L, Vin, sh, on_start);
        else
            split_wave_a<T, true>(md, r0, r_end, col, L, Vin, sh, on_start);
        return false;
    }
    if constexpr (SV::NW == 3) {
        if (wave == 1) return split_wave_c<T, 1>(md, r0, L, Vout, sh);
        return split_wave_c<T, 2>(md, r0, L, Vout, sh);
    } else {
        return split_wave_c<T, 1>(md, r0, L, Vout, sh);
    }
}

// A round of the active schedule with kSplitWaves waves per tile (block 0:
// the round's accounting).  a.wave_stride counts tiles (visiting blocks).
template <int T>
__global__ __launch_bounds__(kSplitThreads) void k_sweep_split(RoundArgs a) {
    // The block's first list entry and the round's count are the start of
    // the round's longest chain of dependent loads: they are issued before
    // anything else (the entry index is clamped into the list; block 0, the
    // accounting block, reads entry 0 and ignores it).
    int i = (int)blockIdx.x - 1;
    const int ie = i >= 0 && i < a.n_tile_ids ? i : 0;
    const uint64_t e0 = __hip_atomic_load(reinterpret_cast<const uint64_t*>(a.list_in + 2 * ie), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
    const int cnt = __hip_atomic_load(a.count_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    // the one maze's description, read while those loads are in flight
    const MazeDev md_one = a.md0;
    const bool one = a.n_slots == 1;
    if (a.round_base) a.round_id += *a.round_base;
    if (blockIdx.x == 0) {
        round_accounting<0, kSplitThreads>(a);
        return;
    }
    __shared__ SplitShared<T> sh;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = lane_id();
    const int stride = a.wave_stride;
    uint64_t e = e0;
    const int n = __builtin_amdgcn_readfirstlane(cnt);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kSplitWaves - 1; ++k) sh.ready[k] = 0;
        sh.done = 0;
    }
    lds_barrier();
    for (; i < n; i += stride) {
        const int g = __builtin_amdgcn_readfirstlane((int)(uint32_t)e);
        const int slot = __builtin_amdgcn_readfirstlane((int)(uint32_t)(e >> 32));
        if (i + stride < n) e = *reinterpret_cast<const uint64_t*>(a.list_in + 2 * (i + stride));
        const MazeDev md = one ? md_one : a.mazes[slot];
        const int lt = g - md.tile_base;
        const int ty = lt / md.tiles_x, tx = lt - ty * md.tiles_x;
        auto on_start = [&]() {
            if (lane == 0) visit_bookkeeping_active(a, g, slot, md, ty, tx);
        };
        // (the runtime selects this kernel for tiles of T rows only)
        const int r0 = ty * T;
        bool changed = false;
        {
            constexpr int TW = kLanes - 2 * T;
            const int col = tx * TW - T + lane;
            const bool col_ok = col >= 0 && col < md.pitch;
            VisitLane L;
            const int cc = col_ok ? col : 0;
            L.voff = cc * 4;
            L.soff = (lane >= T && lane < kLanes - T && col < md.W) ? L.voff : kDroppedStore;
            L.moff = (cc >> 5) * 4;
            L.vrow = md.pitch * 4;
            L.mrow = md.mpitch * 4;
            L.shift = (uint32_t)(col & 31);
            L.col_ok = col_ok;
            L.inner = lane >= T && lane < kLanes - T && col < md.W;
            int32_t* const Vin = a.parity ? md.V[1] : md.V[0];
            int32_t* const Vout = a.parity ? md.V[0] : md.V[1];
            changed = split_visit<T>(wave, md, r0, col, L, Vin, Vout, sh, on_start);
        }
        // the last wave, which knows the result, claims the 3x3 tiles around
        // the tile for the next round and reserves their list entries
        if (wave == kSplitWaves - 1 && changed) {
            const int ny = ty + lane / 3 - 1, nx = tx + lane % 3 - 1;
            const int gn = md.tile_base + ny * md.tiles_x + nx;
            bool won = false;
            if (lane < 9 && ny >= 0 && ny < md.tiles_y && nx >= 0 && nx < md.tiles_x)
                won = atomicExch(&a.flags_out[gn], 1) == 0;
            const uint64_t wmask = __ballot(won);
            const int nwon = __popcll(wmask);
            if (nwon > 0) {
                int base = 0;
                if (lane == 0) base = atomicAdd(a.count_out, nwon);
                base = __builtin_amdgcn_readfirstlane(base);
                if (won) {
                    const int k = base + __popcll(wmask & ((1ull << lane) - 1));
                    a.list_out[2 * k] = gn;
                    a.list_out[2 * k + 1] = slot;
                }
                if (a.n_slots > 1 && lane == 0) atomicAdd(&a.sched_out[slot], nwon);
            }
        }
        // both waves are done with this tile's LDS before it is reset
        lds_barrier();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < kSplitWaves - 1; ++k) sh.ready[k] = 0;
            sh.done = 0;
        }
        lds_barrier();
    }
}

#define OMAP_DEFINE_SWEEP_SPLIT(t) OMAP_DEFINE_SWEEP_SPLIT_(t)
#define OMAP_DEFINE_SWEEP_SPLIT_(t)                                                                   \
    hipError_t launch_sweep_split_T##t(const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0, \
                                       hipEvent_t e1) {                                               \
        RoundArgs b = a;                                                                              \
        b.wave_stride = grid;                                                                         \
        if (e0 != nullptr)                                                                            \
            hipExtLaunchKernelGGL((k_sweep_split<t>), dim3(grid + 1), dim3(kSplitThreads), 0, s, e0, e1, 0, b); \
        else                                                                                          \
            hipLaunchKernelGGL((k_sweep_split<t>), dim3(grid + 1), dim3(kSplitThreads), 0, s, b);     \
        return hipGetLastError();                                                                     \
    }                                                                                                 \
    int sweep_split_blocks_per_cu_T##t() {                                                            \
        int blocks = 0;                                                                               \
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sweep_split<t>, kSplitThreads, 0); \
        return e == hipSuccess ? blocks : 0;                                                          \
    }

}  // namespace omap
