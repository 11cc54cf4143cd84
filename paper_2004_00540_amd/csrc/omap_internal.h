// Internal declarations shared by the device kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omap {

constexpr int kLanes = 64;                          // CDNA wavefront
constexpr int kWavesPerBlock = 4;
constexpr int kBlockThreads = kLanes * kWavesPerBlock;
constexpr uint32_t kObstacleBit = 0x80000000u;      // in-register obstacle marker

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
};

// Per-maze progress states.
enum : int32_t { kMazeIdle = 0, kMazeRunning = 1, kMazeDone = 2 };

// Arguments of one round of the tile schedule.  Round r reads the tile list
// and flags of parity r&1 and appends the tiles to visit in round r+1 to the
// other parity; a tile is appended at most once per round (its flag is set by
// an atomic exchange).
struct RoundArgs {
    const MazeDev* mazes;
    const int32_t* tile_maze;     // global tile id -> maze slot (-1 = unused id)
    int32_t n_tile_ids;           // size of the tile id space
    const int32_t* list_in;       // tiles visited this round
    int32_t* count_in;            // reset to 0 when the round finishes
    int32_t* flags_in;            // cleared as the tiles of this round are visited
    int32_t* list_out;            // tiles scheduled for the next round
    int32_t* count_out;
    int32_t* flags_out;           // 1 = already scheduled for the next round
    int32_t* maze_changed;        // per slot: some tile changed this round
    int32_t* maze_sched;          // per slot: tiles scheduled for the next round
    unsigned long long* maze_sched_cells;  // per slot: their interior cells
    int32_t* maze_state;          // per slot: kMaze*
    int64_t* maze_rounds;         // per slot: rounds with at least one tile visited
    int64_t* maze_visits;         // per slot: tile visits
    int64_t* maze_cell_visits;    // per slot: interior cells of visited tiles
    unsigned long long* total_cells;  // all slots: interior cells of visited tiles
    int32_t n_slots;
    int32_t parity;               // activity buffer read this round
    int32_t tile_rows;            // interior rows per tile
    int32_t tile_cols;            // interior columns per tile (64*C - 2T)
    int32_t dense;                // 1 = dense schedule
};

// ---- launch wrappers (omap_kernels.hip) -------------------------------------
hipError_t launch_pack_mask(const uint8_t* occ, int32_t H, int32_t W, uint32_t* mask,
                            int32_t mpitch, hipStream_t s);
hipError_t launch_fill(int32_t* p, int64_t n_elems, int32_t value, hipStream_t s);
// Seed slot's sources (V := K) and schedule their tiles for the round that
// reads parity a.parity (a.list_in / a.count_in / a.flags_in).
hipError_t launch_seed(const RoundArgs& a, int32_t slot, const int32_t* src_rc, int32_t n_src,
                       int32_t* bad_count, hipStream_t s);
// Schedule every tile of `slot` for the round that reads parity a.parity.
hipError_t launch_schedule_all(const RoundArgs& a, int32_t slot, int32_t n_tiles, hipStream_t s);
hipError_t launch_check_sources(const uint32_t* mask, int32_t mpitch, const int32_t* src_rc,
                                int32_t n_src, int32_t* bad_count, hipStream_t s);
bool sweep_supported(int T, int C);
hipError_t launch_sweep(int T, int C, const RoundArgs& a, int32_t grid, hipStream_t s);
hipError_t launch_finish(const RoundArgs& a, hipStream_t s);
hipError_t launch_slot_reset(const RoundArgs& a, int32_t slot, hipStream_t s);
hipError_t launch_reduce(const MazeDev* mazes, const int32_t* tile_maze, int32_t tile_begin,
                         int32_t tile_end, const int32_t* slot_select, int32_t tile_rows,
                         int32_t tile_cols, int32_t parity, int32_t* maze_min,
                         unsigned long long* maze_reached, hipStream_t s);
hipError_t launch_path_lengths(const MazeDev* mazes, const int32_t* tgt_slot, const int32_t* tgt_rc,
                               int32_t n_tgt, int32_t parity, int32_t* len, hipStream_t s);
hipError_t launch_scan_offsets(const int32_t* len, int32_t n, int64_t* offsets, hipStream_t s);
hipError_t launch_walk(const MazeDev* mazes, const int32_t* tgt_slot, const int32_t* tgt_rc,
                       int32_t n_tgt, int32_t parity, const int32_t* len, const int64_t* offsets,
                       int32_t* cells, hipStream_t s);
hipError_t launch_activity(const MazeDev* mazes, int32_t slot, int32_t H, int32_t W,
                           int32_t parity, int32_t offset, int32_t* dst, int64_t dpitch,
                           hipStream_t s);
hipError_t launch_selftest(int32_t* out, hipStream_t s);
int sweep_max_waves_per_cu(int T, int C);

}  // namespace omap
