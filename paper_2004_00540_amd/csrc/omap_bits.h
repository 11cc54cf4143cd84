// Bit-sliced reached-set propagation (an alternative encoding of the same
// layers, for the active schedule with one launch per round).
//
// With d(x) the 8-neighbour step distance from the nearest source, the layer
// output of the paper is A_L(x) = max(0, L + 1 - d(x)) (Sec. Methods; the
// closed form is what the tests pin), and the integer sweeps hold it as
// V = K - d.  Here the state is instead the reached set R_n = {x : d(x) <= n},
// one bit per cell: R_0 = sources and R_{n+1} = free AND dilate3x3(R_n), so a
// layer costs a few bitwise operations per 32 cells and about 3 bits of
// traffic per cell (R in, free mask, R out) instead of 8.125 bytes.  A cell
// entering R at layer n gets V = K - n written once (4 B per reached cell, in
// activity buffer 0);
// V is then exactly what the integer sweeps produce, and everything after
// propagation (run-time L, copy-out, paths) is shared.
//
// Layer numbers must be exact, so every tile of a maze advances the same T
// layers per round (round r of a maze covers layers (r - round0) T + 1 ..
// + T) from ping-pong bit planes; the active schedule (visit a tile while it
// or a neighbour changed) keeps both planes of an unvisited tile equal, as for
// the integer sweeps.  A wave holds 64 words of a row, 2048 columns, of which
// the outer word on each side is halo (at most 32 layers per visit); tiles are
// tile_rows x 1984 cells.
#pragma once

#include "omap_sweep.h"

namespace omap {

// One row of the bit pipeline: stage s keeps the reached words of its last
// three input rows in r[s][..] and their free masks in f[s][..] (slots rotate
// as in sweep_row).  Stage s emits row i-1-s after s+1 layers into stage s+1's
// slot P; `fresh` receives, per stage, the bits that entered R at that stage.
template <int T, int P, bool GUARD>
__device__ __forceinline__ void bits_row(uint32_t (&r)[T][3], uint32_t (&f)[T][3], uint32_t& out,
                                         uint32_t (&fresh)[T], int smax) {
    constexpr int PA = (P + 1) % 3, PB = (P + 2) % 3;
#pragma unroll
    for (int s = 0; s < T; ++s) {
        fresh[s] = 0;
        if (!GUARD || s <= smax) {
            const uint32_t v = r[s][PA] | r[s][PB] | r[s][P];
            const uint32_t left = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, true);
            const uint32_t right = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, true);
            // column c sees c-1 (bit c-1, or bit 31 of the word to the left) and c+1
            const uint32_t h = v | ((v << 1) | (left >> 31)) | ((v >> 1) | (right << 31));
            const uint32_t o = h & f[s][PB];
            fresh[s] = o ^ r[s][PB];   // o contains the centre row (a subset of free)
            if (s + 1 < T) {
                r[s + 1 < T ? s + 1 : s][P] = o;
                f[s + 1 < T ? s + 1 : s][P] = f[s][PB];
            } else {
                out = o;
            }
        }
    }
}

// Writes V = K - n for the bits of `m` (interior cells of row `row`, word
// `word`) that entered R at layer n, into activity buffer 0 (the one the
// runtime reads for this schedule).
__device__ __forceinline__ void bits_write_v(const MazeDev& md, int row, int word, uint32_t m, int32_t val) {
    int32_t* const v = md.V[0] + (int64_t)row * md.pitch + word * 32;
    while (m != 0) {
        const int b = __builtin_ctz(m);
        m &= m - 1;
        v[b] = val;
    }
}

template <int T, int P, bool GUARD>
__device__ __forceinline__ void bits_iter(uint32_t (&r)[T][3], uint32_t (&f)[T][3], uint32_t& vr, uint32_t& vm,
                                          const MazeDev& md, const uint32_t* Rin, uint32_t* Rout, int R, int r0,
                                          int r_end, int word, bool word_ok, bool inner, int smax, int n0,
                                          uint32_t& chg) {
    const bool ok = R >= 0 && R < md.H && word_ok;
    r[0][P] = ok ? vr : 0u;
    f[0][P] = ok ? ~vm : 0u;   // guard bits (columns >= W) are obstacles
    {
        const int Rn = min(max(R + 3, 0), md.H - 1);
        const int64_t x = (int64_t)Rn * md.mpitch + (word_ok ? word : 0);
        vr = *(const __attribute__((address_space(1))) uint32_t*)(Rin + x);
        vm = *(const __attribute__((address_space(1))) uint32_t*)(md.mask + x);
    }
    uint32_t out = 0;
    uint32_t fresh[T];
    bits_row<T, P, GUARD>(r, f, out, fresh, smax);
    if (inner) {
        // stage s emitted row R - 1 - s: record the cells that entered R there
#pragma unroll
        for (int s = 0; s < T; ++s) {
            const int row = R - 1 - s;
            const int n = n0 + s + 1;
            if (row >= r0 && row < r_end && fresh[s] != 0) {
                chg |= fresh[s];
                if (n < md.K) bits_write_v(md, row, word, fresh[s], md.K - n);
            }
        }
        const int Ro = R - T;
        if (Ro >= r0 && Ro < r_end) Rout[(int64_t)Ro * md.mpitch + word] = out;
    }
}

// T layers of the reached set on one tile.  Returns true (wave-uniform) if
// any interior cell entered R.
template <int T>
__device__ bool bits_tile(const MazeDev& md, int ty, int tx, int tile_rows, int parity, int n0) {
    const int lane = lane_id();
    const int r0 = ty * tile_rows;
    const int r_end = min(r0 + tile_rows, md.H);
    const int word = tx * (kLanes - 2) - 1 + lane;   // one halo word on each side
    const bool word_ok = word >= 0 && word < md.mpitch;
    const bool inner = lane >= 1 && lane < kLanes - 1 && word_ok;
    const uint32_t* Rin = parity ? md.R[1] : md.R[0];
    uint32_t* Rout = parity ? md.R[0] : md.R[1];

    uint32_t r[T][3], f[T][3];
#pragma unroll
    for (int s = 0; s < T; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            r[s][k] = 0;
            f[s][k] = 0;
        }
    uint32_t chg = 0;
    const int n_iter = (r_end - r0) + 2 * T;
    uint32_t vr0, vm0, vr1, vm1, vr2, vm2;
    {
        const int wc = word_ok ? word : 0;
        const int a = min(max(r0 - T, 0), md.H - 1), b = min(max(r0 - T + 1, 0), md.H - 1),
                  c = min(max(r0 - T + 2, 0), md.H - 1);
        vr0 = Rin[(int64_t)a * md.mpitch + wc];
        vm0 = md.mask[(int64_t)a * md.mpitch + wc];
        vr1 = Rin[(int64_t)b * md.mpitch + wc];
        vm1 = md.mask[(int64_t)b * md.mpitch + wc];
        vr2 = Rin[(int64_t)c * md.mpitch + wc];
        vm2 = md.mask[(int64_t)c * md.mpitch + wc];
    }
    // the first 2T steps skip the stages no stored row needs (see sweep_tile)
    constexpr int kWarm = 3 * ((2 * T + 2) / 3);
    int i = 0;
#pragma unroll 1
    for (; i < kWarm; i += 3) {
        const int R = r0 - T + i;
        bits_iter<T, 0, true>(r, f, vr0, vm0, md, Rin, Rout, R, r0, r_end, word, word_ok, inner, (i >> 1) - 1, n0, chg);
        bits_iter<T, 1, true>(r, f, vr1, vm1, md, Rin, Rout, R + 1, r0, r_end, word, word_ok, inner,
                              ((i + 1) >> 1) - 1, n0, chg);
        bits_iter<T, 2, true>(r, f, vr2, vm2, md, Rin, Rout, R + 2, r0, r_end, word, word_ok, inner,
                              ((i + 2) >> 1) - 1, n0, chg);
    }
#pragma unroll 1
    for (; i < n_iter; i += 3) {
        const int R = r0 - T + i;
        bits_iter<T, 0, false>(r, f, vr0, vm0, md, Rin, Rout, R, r0, r_end, word, word_ok, inner, 0, n0, chg);
        bits_iter<T, 1, false>(r, f, vr1, vm1, md, Rin, Rout, R + 1, r0, r_end, word, word_ok, inner, 0, n0, chg);
        bits_iter<T, 2, false>(r, f, vr2, vm2, md, Rin, Rout, R + 2, r0, r_end, word, word_ok, inner, 0, n0, chg);
    }
    return __ballot(chg != 0) != 0;
}

// One round of the bit-sliced propagation over the listed tiles (active
// schedule), with the next round's claims reserved per block as in
// sweep_round.  A maze whose rounds have covered every layer below K is not
// visited any more.
template <int T>
__global__ __launch_bounds__(kBlockThreads) void k_bits(RoundArgs a) {
    // first list entry and count issued before anything else (see k_sweep)
    int i = ((int)blockIdx.x - 1) * kWavesPerBlock + (int)(threadIdx.x >> 6);   // block 0: the accounting block
    const int ie = i >= 0 && i < a.n_tile_ids ? i : 0;
    uint64_t e = __hip_atomic_load(reinterpret_cast<const uint64_t*>(a.list_in + 2 * ie), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    const int cnt = __hip_atomic_load(a.count_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (a.round_base) a.round_id += *a.round_base;
    if (blockIdx.x == 0) {   // the accounting block (see k_sweep)
        round_accounting<T>(a);
        return;
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = lane_id();
    const int stride = a.wave_stride;
    const int n = __builtin_amdgcn_readfirstlane(cnt);
    __shared__ int s_cnt[2][kWavesPerBlock];
    __shared__ int s_base[2];
    int par = 0;
    for (int ib = (blockIdx.x - 1) * kWavesPerBlock; ib < n; ib += stride, par ^= 1) {
        i = ib + wave;
        int slot = 0, gn = 0, g = 0, ty = 0, tx = 0;
        bool won = false, visited = false;
        MazeDev md;
        if (i < n) {
            g = __builtin_amdgcn_readfirstlane((int)(uint32_t)e);
            slot = __builtin_amdgcn_readfirstlane((int)(uint32_t)(e >> 32));
            if (i + stride < n) e = *reinterpret_cast<const uint64_t*>(a.list_in + 2 * (i + stride));
            md = a.n_slots == 1 ? a.md0 : a.mazes[slot];
            const int64_t n0 = (int64_t)(a.round_id - md.round0) * T;   // layers done before this round
            if (n0 + 1 < md.K) {
                const int lt = g - md.tile_base;
                ty = lt / md.tiles_x;
                tx = lt - ty * md.tiles_x;
                visited = true;
                if (bits_tile<T>(md, ty, tx, a.tile_rows, a.parity, (int)n0)) {
                    const int ny = ty + lane / 3 - 1, nx = tx + lane % 3 - 1;
                    gn = md.tile_base + ny * md.tiles_x + nx;
                    if (lane < 9 && ny >= 0 && ny < md.tiles_y && nx >= 0 && nx < md.tiles_x)
                        won = atomicExch(&a.flags_out[gn], 1) == 0;
                }
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
        if (i < n && lane == 0) {
            if (visited) visit_bookkeeping_active(a, g, slot, md, ty, tx);
            else a.flags_in[g] = 0;
        }
    }
}

#define OMAP_DEFINE_BITS_VARIANT(t) OMAP_DEFINE_BITS_VARIANT_(t)
#define OMAP_DEFINE_BITS_VARIANT_(t)                                                                  \
    hipError_t launch_bits_T##t(const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0,       \
                                hipEvent_t e1) {                                                      \
        RoundArgs b = a;                                                                              \
        b.wave_stride = grid * kWavesPerBlock;                                                        \
        if (e0 != nullptr)                                                                            \
            hipExtLaunchKernelGGL((k_bits<t>), dim3(grid + 1), dim3(kBlockThreads), 0, s, e0, e1, 0, b); \
        else                                                                                          \
            hipLaunchKernelGGL((k_bits<t>), dim3(grid + 1), dim3(kBlockThreads), 0, s, b);           \
        return hipGetLastError();                                                                     \
    }                                                                                                 \
    int bits_blocks_per_cu_T##t() {                                                                   \
        int blocks = 0;                                                                               \
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_bits<t>, kBlockThreads, 0) ==  \
                       hipSuccess                                                                     \
                   ? blocks                                                                           \
                   : 0;                                                                               \
    }

}  // namespace omap
