// Internal declarations shared by the device kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omap {

constexpr int kLanes = 64;                          // CDNA wavefront
constexpr int kWavesPerBlock = 4;
constexpr int kBlockThreads = kLanes * kWavesPerBlock;
constexpr uint32_t kObstacleBit = 0x80000000u;      // in-register obstacle marker
// Visit counters are kept in kSpread copies (a block adds to copy blockIdx mod
// kSpread) so that concurrent waves do not serialise on one address; readers
// sum the copies.
constexpr int kSpread = 16;
// Interior columns of a bit-sliced tile: 64 lanes x 32 bits minus one halo
// word on each side.
constexpr int kBitsTileColumns = (kLanes - 2) * 32;

// Maze state on the device.  Activity rows are `pitch` int32 apart (pitch a
// multiple of 64, so rows are 256-byte aligned); the obstacle mask has one bit
// per cell (bit c&31 of word c>>5 of the row, 1 = obstacle), `mpitch` words per
// row, and the bits of columns >= W are set (guard bits).
struct MazeDev {
    int32_t H, W;
    int32_t pitch;
    int32_t mpitch;
    int32_t tiles_x, tiles_y;
    int32_t tile_base;      // global id of tile (0, 0)
    int32_t K;              // source level of the encoding
    int32_t* V[2];          // activity ping-pong
    const uint32_t* mask;
    uint32_t* R[2];         // bit-sliced schedule: reached-set planes (mask layout), else null
    int32_t round0;         // bit-sliced schedule: index of the maze's first round
};

// Arguments of round r of the tile schedule.  The tile lists and their dedup
// flags alternate by r mod 2; the list counts, the per-maze scheduled counts
// and the dense schedule's "changed" flags rotate over three buffers by r mod
// 3, so that round r can clear the buffer round r+1 will fill without racing
// with anything that reads or writes during round r.
struct RoundArgs {
    const MazeDev* mazes;
    const int32_t* tile_maze;     // global tile id -> maze slot (-1 = unused id)
    int32_t n_tile_ids;           // size of the tile id space
    const int32_t* list_in;       // (tile id, slot) pairs of round r (active schedule)
    const int32_t* count_in;      // their number
    int32_t* flags_in;            // cleared as the tiles of round r are visited
    int32_t* list_out;            // (tile id, slot) pairs scheduled for round r+1
    int32_t* count_out;           // their number (dense: 1 = some tile changed)
    int32_t* flags_out;           // 1 = already scheduled for round r+1
    int32_t* count_clear;         // count of round r+2, zeroed by round r
    const int32_t* sched_in;      // per slot: tiles scheduled for round r (more than one slot)
    int32_t* sched_out;           // per slot: tiles scheduled for round r+1 (kept only with
                                  // more than one slot; with one slot it equals *count_out)
    int32_t* sched_clear;         // per slot: scheduled counts of round r+2, zeroed by round r
    int32_t* dchg_prev;           // dense, per slot: changed in round r-1 (visit in round r)
    int32_t* dchg_cur;            // dense, per slot: changed in round r
    int32_t* dchg_clear;          // dense, per slot: flags of round r+1, zeroed by round r
    int32_t* maze_last_round;     // per slot: last round with a tile visited
    uint8_t* touched;             // per tile id: written since its maze's buffers were last cleared
    int64_t* maze_visits;         // [slot][kSpread]: tile visits
    int64_t* maze_cell_visits;    // [slot][kSpread]: interior cells of visited tiles
    unsigned long long* total_cells;  // [kSpread], all slots: interior cells of visited tiles
    int32_t n_slots;
    int32_t round_id;             // r (wraps; only differences are used); in a graph replay
                                  // the round's offset in the captured group
    const int32_t* round_base;    // graph replays: device counter holding the group's first
                                  // round, added to round_id by the kernels (else null)
    int32_t parity;               // activity buffer read in round r (r mod 2)
    int32_t tile_rows;            // interior rows per tile
    int32_t tile_cols;            // interior columns per tile (64*C - 2T)
    int32_t dense;                // 1 = dense schedule
    int32_t wave_stride;          // waves in the launch (set by the launch wrapper)
    MazeDev md0;                  // copy of mazes[0] when n_slots == 1 (saves a dependent load)
};

// Sweep variants (layers per visit T, columns per lane C); each is compiled in
// its own translation unit (omap_sweep_variant.hip with OMAP_T, OMAP_C).
#define OMAP_SWEEP_VARIANTS(X) \
    X(4, 4) X(8, 4) X(12, 4) X(16, 4) X(4, 2) X(8, 2) X(12, 2) X(16, 2) X(24, 2) X(32, 2) \
    X(4, 1) X(8, 1) X(12, 1) X(16, 1)

#define X(t, c)                                                                                       \
    hipError_t launch_sweep_T##t##_C##c(const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0, \
                                        hipEvent_t e1);                                               \
    int sweep_blocks_per_cu_T##t##_C##c();
OMAP_SWEEP_VARIANTS(X)
#undef X

// Two-wave visits (omap_sweep_split.h): one column per lane, 16 layers per
// visit, tiles of 16 rows; defined in the T = 16, C = 1 sweep variant.
hipError_t launch_sweep_split_T16(const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
int sweep_split_blocks_per_cu_T16();

// Bit-sliced variants (layers per visit); omap_bits_variant.hip with OMAP_BITS_T.
#define OMAP_BITS_VARIANTS(X) X(8) X(16)

#define X(t)                                                                                          \
    hipError_t launch_bits_T##t(const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1); \
    int bits_blocks_per_cu_T##t();
OMAP_BITS_VARIANTS(X)
#undef X

// ---- launch wrappers (omap_kernels.hip) -------------------------------------
hipError_t launch_pack_mask(const uint8_t* occ, int32_t H, int32_t W, uint32_t* mask,
                            int32_t mpitch, hipStream_t s);
hipError_t launch_fill(int32_t* p, int64_t n_elems, int32_t value, hipStream_t s);
// Seed slot's sources (V := K) and schedule their tiles into a.list_out /
// a.count_out / a.flags_out / a.sched_out (the runtime points these at the
// round about to run).
// (src_slot: per-source slots, or nullptr for `slot`)
hipError_t launch_seed(const RoundArgs& a, int32_t slot, const int32_t* src_rc, const int32_t* src_slot,
                       int32_t n_src, int32_t* bad_count, hipStream_t s);
hipError_t launch_check_sources(const uint32_t* mask, int32_t mpitch, const int32_t* src_rc,
                                int32_t n_src, int32_t* bad_count, hipStream_t s);
bool sweep_supported(int T, int C);
// e0 / e1 (optional, both or neither): events that record the kernel's own
// start and end (hipExtLaunchKernel), for profiling.
hipError_t launch_sweep(int T, int C, const RoundArgs& a, int32_t grid, hipStream_t s,
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Clears slot's counters before its seeds (last round = r-1; dense: marks the
// maze for a visit in the round about to run through a.dchg_prev).
bool bits_supported(int T);
int bits_max_waves_per_cu(int T);
hipError_t launch_bits(int T, const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
hipError_t launch_slot_reset(const RoundArgs& a, const int32_t* slots, int32_t n, hipStream_t s);

// Packing of several mazes' occupancy in one launch.
struct PackJob {
    const uint8_t* occ;
    uint32_t* mask;
    int32_t H, W, mpitch;
    int64_t word_begin;   // first word of this maze in the concatenation
};
hipError_t launch_pack_mask_many(const PackJob* jobs, int32_t n_jobs, int64_t total_words, hipStream_t s);
hipError_t launch_check_sources_many(const MazeDev* mazes, const int32_t* src_rc, const int32_t* src_slot,
                                     int32_t n, int32_t* bad, hipStream_t s);
// Smallest positive activity and reached count of the touched tiles in
// [tile_begin, tile_end) of the selected slots.
hipError_t launch_reduce(const MazeDev* mazes, const int32_t* tile_maze, const uint8_t* touched,
                         int32_t tile_begin, int32_t tile_end, const int32_t* slot_select, int32_t tile_rows,
                         int32_t tile_cols, int32_t parity, int32_t* maze_min,
                         unsigned long long* maze_reached, hipStream_t s);
hipError_t launch_path_lengths(const MazeDev* mazes, const int32_t* tgt_slot, const int32_t* tgt_rc,
                               int32_t n_tgt, int32_t parity, int32_t* len, hipStream_t s);
// order (optional): receives the targets by path length, longest first
hipError_t launch_scan_offsets(const int32_t* len, int32_t n, int64_t* offsets, hipStream_t s,
                               int32_t* order = nullptr);
// order (optional): the walk's order of the targets (from launch_scan_offsets)
hipError_t launch_walk(const MazeDev* mazes, const int32_t* tgt_slot, const int32_t* tgt_rc,
                       int32_t n_tgt, int32_t parity, const int32_t* len, const int64_t* offsets,
                       int32_t* cells, hipStream_t s, const int32_t* order = nullptr);
hipError_t launch_walk_random(const MazeDev* mazes, const int32_t* tgt_slot, const int32_t* tgt_rc,
                              const int32_t* tgt_local, int32_t n_tgt, int32_t parity, uint64_t seed,
                              const int32_t* len, const int64_t* offsets, int32_t* cells, hipStream_t s);
hipError_t launch_walk_euclid(bool write, const MazeDev* mazes, const int32_t* tgt_slot,
                              const int32_t* tgt_rc, int32_t n_tgt, int32_t parity, int32_t* len,
                              const int64_t* offsets, int32_t* cells, hipStream_t s);
hipError_t launch_source_index(const MazeDev* mazes, const int32_t* tgt_slot, int32_t n_tgt,
                               const int32_t* len, const int64_t* offsets, const int32_t* cells,
                               const int32_t* src_sorted, const int32_t* src_base, const int32_t* src_n,
                               int32_t* out, hipStream_t s);
hipError_t launch_activity(const MazeDev* mazes, int32_t slot, int32_t H, int32_t W,
                           int32_t parity, int32_t offset, int32_t* dst, int64_t dpitch,
                           hipStream_t s);
hipError_t launch_selftest(int32_t* out, hipStream_t s);
// *counter += add (one thread): advances the round counter of graph replays.
hipError_t launch_round_advance(int32_t* counter, int32_t add, hipStream_t s);
// Zeroes both activity buffers (and bit planes) over the interiors of the
// touched tiles among tile ids [tile_begin, +n_tiles) of the selected mazes
// (sel == nullptr: all) and clears their touched flags.
hipError_t launch_clear_touched(const RoundArgs& a, int32_t tile_begin, int32_t n_tiles, const int32_t* sel,
                                hipStream_t s);
int sweep_max_waves_per_cu(int T, int C);

}  // namespace omap

#include "omap.h"

namespace omap {

// Records `message` as the thread's last error (omap_last_error) and returns st.
omap_status_t report_error(omap_status_t st, const char* message);

}  // namespace omap
