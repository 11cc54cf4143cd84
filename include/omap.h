/*
 * omap.h -- C ABI of the MI355X (gfx950) oMAP maze planner.
 *
 * Method: Kulvicius, Herzog, Tamosiunaite, Woergoetter, "Generation of Paths in
 * a Maze using a Deep Network without Learning" (arXiv 2004.00540).
 *
 * The problem (Sec. Methods, "Input"): an m x n grid environment with
 * obstacles, s >= 1 source cells and any number of target cells.  The network
 * (Sec. Methods, "Activity Map Generation"; Fig. net) is L identical layers of
 * 3x3 / stride-1 / zero-padded max pooling, a sum with the environment map I_e
 * (0 free, -maxint obstacle) and the source map I_s (1 at sources), and a
 * rectifier; its output is the activity map O.  A path from each target to its
 * closest source is read back by repeatedly stepping to the 8-neighbour of
 * largest activity (Sec. "Path Reconstruction", simple path reconstruction).
 *
 * Conventions for every call:
 *   - Grids are row-major; cell (r, c) has linear index r*width + c.
 *   - Occupancy is uint8, nonzero = obstacle.
 *   - Coordinates are int32 (row, col) pairs, host memory.
 *   - "_dev" pointers are device (HBM) pointers owned by the caller; "_host"
 *     pointers are host pointers owned by the caller.  The library never keeps
 *     a caller pointer past the call that received it.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Device work is
 *     ordered on that stream; calls documented as synchronous wait for it.
 *   - Every call returns a status; out-parameters are written only on OMAP_OK
 *     unless stated otherwise.  omap_last_error() gives a thread-local message
 *     for the most recent failure.
 *   - Sizes: height, width >= 1 and height*width < 2^31.
 *
 * Readings of the paper fixed by this interface:
 *   - Layers: max_layers = L >= 0 runs the L-layer network; the activity before
 *     the first layer is I_s, so after layer n every source holds n+1 (Sec.
 *     Methods).  max_layers = OMAP_AUTO_LAYERS determines L at run time (Sec.
 *     "Determining the number of layers L"): layers are added until the set of
 *     nonzero cells stops growing; the output is the map after the last layer
 *     that grew it (L* = the largest step distance from a source).
 *   - Neighbourhood: the 3x3 window, so moves between diagonal neighbours are
 *     allowed even when both cells beside the diagonal are obstacles.
 *   - Sources must lie on free cells (a source on an obstacle is rejected:
 *     the literal layer would leave a plateau of ones around it).
 *   - Ties in the path walk are broken by the fixed neighbour order
 *     (-1,-1) (-1,0) (-1,+1) (0,-1) (0,+1) (+1,-1) (+1,0) (+1,+1), first
 *     maximum wins (the paper picks at random; every choice has the same
 *     number of steps).
 *   - A target whose activity is 0 (obstacle, unreachable, or farther than L
 *     steps) has no path: its length is -1 and it occupies no cells.
 */
#ifndef OMAP_H
#define OMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum omap_status {
    OMAP_OK = 0,
    OMAP_ERR_INVALID_ARG = 1,          /* NULL pointer, size < 1, bad option value  */
    OMAP_ERR_TOO_LARGE = 2,            /* height*width >= 2^31, or L+1 > 2^31-1     */
    OMAP_ERR_SOURCE_OUT_OF_BOUNDS = 3,
    OMAP_ERR_SOURCE_ON_OBSTACLE = 4,
    OMAP_ERR_NO_SOURCES = 5,
    OMAP_ERR_TARGET_OUT_OF_BOUNDS = 6,
    OMAP_ERR_NOT_PROPAGATED = 7,       /* activity or paths asked before propagate  */
    OMAP_ERR_BUFFER_TOO_SMALL = 8,     /* path cell buffer below cells_needed       */
    OMAP_ERR_OUT_OF_MEMORY = 9,
    OMAP_ERR_HIP = 10,                 /* a HIP runtime call failed                 */
    OMAP_ERR_NOT_FOUND = 11,           /* unknown query id (serving engine)         */
    OMAP_ERR_BUSY = 12                 /* query not finished yet (serving engine)   */
} omap_status_t;

#define OMAP_AUTO_LAYERS (-1)

/* Schedules of tile visits (see omap_options.schedule). */
#define OMAP_SCHEDULE_DEFAULT 0  /* plan: ACTIVE; batch and engine: BITS (the fastest measured for */
                                 /* each; with lane_columns set, or a depth BITS lacks: ACTIVE)   */
#define OMAP_SCHEDULE_ACTIVE 1   /* visit a tile only while it or a neighbour changed             */
#define OMAP_SCHEDULE_DENSE 2    /* visit every tile of a maze until the maze stops changing      */
#define OMAP_SCHEDULE_BITS 3     /* active schedule on a bit-packed reached set instead of int32  */
                                 /* activity: same results; temporal_depth 8 or 16, lane_columns 0 */

/* Round launches (see omap_options.round_launch). */
#define OMAP_LAUNCH_PER_ROUND 0  /* one kernel launch per round, enqueued by the host             */
#define OMAP_LAUNCH_GRAPH 1      /* groups of rounds captured once in a HIP graph and replayed     */

/* Execution options.  Zero-initialised = tuned defaults.  No option changes a
 * result: activity maps and paths are identical bit for bit for every value. */
typedef struct omap_options {
    int32_t temporal_depth;  /* layers applied per tile visit: 4, 8, 12, 16 (and 24, 32    */
                             /* with lane_columns = 2; bit-sliced: 8, 16); 0 = default     */
                             /* (16; active with more than one column per lane: 12)        */
    int32_t tile_rows;       /* interior rows per tile, even, 2..4096, >= temporal_depth;  */
                             /* 0 = default (plan, active, 1 column per lane: depth;       */
                             /* other active and bit-sliced: max(16, depth); dense: 256)   */
    int32_t schedule;        /* OMAP_SCHEDULE_*                                             */
    int32_t check_interval;  /* rounds between host reads of the convergence count;        */
                             /* 0 = adaptive                                                */
    int32_t lane_columns;    /* columns each lane owns (tile strip = 64 x this): 1, 2 or   */
                             /* 4 (1: temporal_depth 4..16); 0 = default (plan, active: 1; */
                             /* batch, engine: 2; dense: 4; the narrowest with the depth)  */
    int32_t round_launch;    /* OMAP_LAUNCH_PER_ROUND (default) or OMAP_LAUNCH_GRAPH        */
} omap_options;

/* The options a plan created with `options` (NULL = all defaults) would run
 * with: every zero field replaced by its default (batches and engines default
 * to other depth / column values, see above).  Host only, no device call.
 * Returns OMAP_ERR_INVALID_ARG (and leaves *resolved untouched) for the same
 * option values the create calls reject. */
omap_status_t omap_resolve_options(const omap_options *options, omap_options *resolved);

/* Per-maze report of a propagation. */
typedef struct omap_propagate_info {
    int64_t layers;           /* L (fixed) or L* (run-time determined)               */
    int64_t sweeps_executed;  /* layers applied by the kernels (>= layers + 1 when   */
                              /* converged: the last visit confirms the fixpoint)    */
    int64_t rounds;           /* temporal blocks in which the maze had tiles visited */
    int64_t tile_visits;      /* tile visits summed over rounds                       */
    int64_t reached_cells;    /* cells with activity > 0                              */
} omap_propagate_info;

/* ---------------------------------------------------------------------------
 * Single maze
 * ------------------------------------------------------------------------- */
typedef struct omap_plan_s *omap_plan_t;

/* Create a plan for one maze (Sec. Methods, "Input"): packs the occupancy into
 * the plan's obstacle bit mask and stores sources and targets.
 *   occupancy_dev  height*width uint8, row-major, nonzero = obstacle (device)
 *   sources_host   n_sources (row, col) pairs, n_sources >= 1, free cells
 *   targets_host   n_targets (row, col) pairs, n_targets >= 0 (NULL if 0)
 *   opts           NULL = defaults
 * Synchronous: on return every input may be freed.  Errors: INVALID_ARG,
 * TOO_LARGE, NO_SOURCES, SOURCE_OUT_OF_BOUNDS, SOURCE_ON_OBSTACLE,
 * TARGET_OUT_OF_BOUNDS, OUT_OF_MEMORY, HIP. */
omap_status_t omap_plan_create(omap_plan_t *out, int32_t height, int32_t width,
                               const uint8_t *occupancy_dev,
                               const int32_t *sources_host, int32_t n_sources,
                               const int32_t *targets_host, int32_t n_targets,
                               const omap_options *opts, void *stream);

/* Replace the occupancy, sources and targets of an existing plan with a new
 * problem of the same height and width, reusing its device buffers.  Same
 * arguments, validation and synchrony as omap_plan_create. */
omap_status_t omap_plan_load(omap_plan_t plan, const uint8_t *occupancy_dev,
                             const int32_t *sources_host, int32_t n_sources,
                             const int32_t *targets_host, int32_t n_targets);

/* Run the network (Sec. Methods, "Activity Map Generation"; Sec. "Determining
 * the number of layers L").
 *   max_layers  L >= 0 with L+1 <= 2^31-1, or OMAP_AUTO_LAYERS
 *   info        NULL: asynchronous on the plan's stream (only a few small
 *               host reads of the convergence count);
 *               non-NULL: synchronous, filled on return.
 * Errors: INVALID_ARG, TOO_LARGE, HIP. */
omap_status_t omap_propagate(omap_plan_t plan, int64_t max_layers, omap_propagate_info *info);

/* Copy the activity map O (the network output A_L, Sec. Methods) to
 *   dst_dev: height rows of width int32, row stride dst_pitch_elems >= width.
 * Stream-ordered.  Errors: INVALID_ARG, NOT_PROPAGATED, HIP. */
omap_status_t omap_get_activity(omap_plan_t plan, int32_t *dst_dev, int64_t dst_pitch_elems);

/* Simple path reconstruction (Sec. "Path Reconstruction") from every target.
 *   len_dev      n_targets int32: steps of each path, -1 = no path
 *   offsets_dev  n_targets+1 int64: path k occupies cells[offsets[k] .. offsets[k+1])
 *   cells_dev    linear cell indices r*width + c, target first, source last
 *   cells_capacity  size of cells_dev in elements
 *   cells_needed_host  always written (on OK and on BUFFER_TOO_SMALL)
 * When cells_capacity < cells_needed (or cells_dev is NULL and cells_needed
 * > 0), only cells_needed is written and BUFFER_TOO_SMALL returned; a NULL
 * cells_dev is accepted when no target has a path.  Synchronous.
 * Errors: INVALID_ARG, NOT_PROPAGATED, BUFFER_TOO_SMALL, HIP. */
omap_status_t omap_extract_paths(omap_plan_t plan, int32_t *len_dev, int64_t *offsets_dev,
                                 int32_t *cells_dev, int64_t cells_capacity,
                                 int64_t *cells_needed_host);

/* Path reconstruction variants (Sec. "Path Reconstruction"). */
#define OMAP_WALK_FIRST_MAX 0     /* simple reconstruction, ties by the fixed neighbour order  */
#define OMAP_WALK_RANDOM_TIES 1   /* simple reconstruction, the paper's random choice among     */
                                  /* maximal neighbours, made reproducible: at move s of target */
                                  /* t the choice is SplitMix64out(seed ^ (t << 32) ^ s) mod the */
                                  /* number of maxima, maxima listed in the fixed order         */
#define OMAP_WALK_EUCLIDEAN 2     /* Euclidean reconstruction (Eq. 1): climb through 4-neighbours */
                                  /* (first maximum in the order up, left, right, down), at most */
                                  /* one sideways move to an equal 4-neighbour per activity      */
                                  /* level, else the first maximal 8-neighbour; then remove each */
                                  /* point whose neighbours on the path are diagonal neighbours */
                                  /* (one left-to-right pass).  len = segments of the result.    */

typedef struct omap_walk_options {
    int32_t mode;      /* OMAP_WALK_* */
    int32_t reserved;  /* 0 */
    uint64_t seed;     /* OMAP_WALK_RANDOM_TIES only */
} omap_walk_options;

/* omap_extract_paths with a reconstruction variant (walk NULL = FIRST_MAX)
 * and, when source_index_dev is not NULL, n_targets int32 receiving the index
 * in the source list of the source each path ends on (its closest source,
 * first listed if repeated; -1 for no path) -- the paper's taxi assignment
 * (Sec. "Multi-source Multi-target Path Planning").  Same synchrony and
 * errors as omap_extract_paths. */
omap_status_t omap_extract_paths_ex(omap_plan_t plan, const omap_walk_options *walk,
                                    int32_t *len_dev, int64_t *offsets_dev, int32_t *cells_dev,
                                    int64_t cells_capacity, int64_t *cells_needed_host,
                                    int32_t *source_index_dev);

/* omap_extract_paths for callers that cannot allocate memory: code under HIP
 * graph capture, serving loops and harnesses that forbid allocation.  Same
 * arguments, outputs, errors and synchrony as omap_extract_paths, but the
 * call allocates nothing: the per-target staging (slot ids and target
 * coordinates, 12 bytes per target) lives in a fixed array of
 * 3 * OMAP_NOALLOC_MAX_TARGETS int32 (3 MiB) that the library holds on each
 * device it runs on until the process ends; lengths and offsets go straight
 * to len_dev / offsets_dev.  More than OMAP_NOALLOC_MAX_TARGETS targets:
 * OMAP_ERR_TOO_LARGE.  Every call on one device shares that array and leaves
 * its contents behind: calls that overlap on one device (from several host
 * threads or streams) race, so the caller must serialise them. */
#define OMAP_NOALLOC_MAX_TARGETS (1 << 18)
omap_status_t omap_extract_paths_noalloc(omap_plan_t plan, int32_t *len_dev, int64_t *offsets_dev,
                                         int32_t *cells_dev, int64_t cells_capacity,
                                         int64_t *cells_needed_host);

/* Release the plan and its device buffers.  NULL is a no-op. */
omap_status_t omap_plan_destroy(omap_plan_t plan);

/* ---------------------------------------------------------------------------
 * Batched form: many independent mazes of different sizes advanced together
 * by the same kernel launches (the paper treats one maze per run; each maze's
 * results are those of solving it alone).
 * ------------------------------------------------------------------------- */
typedef struct omap_maze_desc {
    int32_t height, width;
    const uint8_t *occupancy_dev;   /* height*width uint8, nonzero = obstacle (device) */
    const int32_t *sources_host;    /* n_sources (row, col) pairs                      */
    int32_t n_sources;
    const int32_t *targets_host;    /* n_targets (row, col) pairs                      */
    int32_t n_targets;
} omap_maze_desc;

typedef struct omap_batch_s *omap_batch_t;

/* Create a batch of n_mazes >= 1 mazes; validation as omap_plan_create, per
 * maze (the first failing maze's status is returned and omap_last_error()
 * names its index).  Synchronous. */
omap_status_t omap_batch_create(omap_batch_t *out, const omap_maze_desc *mazes, int32_t n_mazes,
                                const omap_options *opts, void *stream);

/* Run every maze: max_layers_host[i] per maze (NULL = all OMAP_AUTO_LAYERS);
 * infos_host: n_mazes reports (NULL = asynchronous). */
omap_status_t omap_batch_propagate(omap_batch_t batch, const int64_t *max_layers_host,
                                   omap_propagate_info *infos_host);

/* Activity map of maze `index`, as omap_get_activity. */
omap_status_t omap_batch_get_activity(omap_batch_t batch, int32_t index, int32_t *dst_dev,
                                      int64_t dst_pitch_elems);

/* Paths of every target of every maze, concatenated in maze order then target
 * order (total = sum of n_targets); layout as omap_extract_paths, with cell
 * indices local to each maze.  Synchronous. */
omap_status_t omap_batch_extract_paths(omap_batch_t batch, int32_t *len_dev, int64_t *offsets_dev,
                                       int32_t *cells_dev, int64_t cells_capacity,
                                       int64_t *cells_needed_host);

/* omap_batch_extract_paths with a reconstruction variant and source indices
 * (per maze: t and the source list are those of the target's own maze). */
omap_status_t omap_batch_extract_paths_ex(omap_batch_t batch, const omap_walk_options *walk,
                                          int32_t *len_dev, int64_t *offsets_dev, int32_t *cells_dev,
                                          int64_t cells_capacity, int64_t *cells_needed_host,
                                          int32_t *source_index_dev);

omap_status_t omap_batch_destroy(omap_batch_t batch);

/* ---------------------------------------------------------------------------
 * Serving form: a request loop with continuous batching.  Queries are copied
 * in at submit; they are admitted into the running set of mazes when a slot
 * and device memory (within memory_budget_bytes) are free, advanced together
 * with every other admitted query, and retired with their paths as soon as
 * they converge, freeing memory for waiting queries.  The results of a query
 * are those of solving it alone with a plan (the paper treats one maze per
 * run; the tests compare both).
 *
 * The engine's host side does not wait for the device while there is device
 * work to enqueue: occupancy grids are copied to pinned memory at submit and
 * reach the device by DMA on a second stream while the rounds run (a query
 * is packed and started at the step after its upload completed), convergence
 * is read from counts copied after each step (one step late), and a
 * retirement runs in three phases across steps (finalize and path lengths on
 * the rounds' stream; walk and copies on the second stream; hand-over).  A
 * step blocks only to stay at most two steps of rounds ahead of the device,
 * or, when nothing is left to advance, until the work in flight completes.
 * ------------------------------------------------------------------------- */
typedef struct omap_engine_s *omap_engine_t;

#define OMAP_QUERY_QUEUED 0
#define OMAP_QUERY_RUNNING 1
#define OMAP_QUERY_DONE 2
#define OMAP_QUERY_FAILED 3

/* Flags of omap_engine_submit_ex. */
#define OMAP_QUERY_KEEP_ACTIVITY 1u   /* keep the query's activity map O (Sec. Methods, "Activity  */
                                      /* Map Generation") for omap_engine_fetch_activity; costs a  */
                                      /* device-to-host copy of height*width int32 at retirement   */

/* max_slots: most queries resident at once; memory_budget_bytes: device bytes
 * the engine may hold for query state (activity, masks, paths). */
omap_status_t omap_engine_create(omap_engine_t *out, int64_t memory_budget_bytes,
                                 int32_t max_slots, const omap_options *opts, void *stream);

/* Queue a query.  occupancy_host: height*width uint8 (host, copied);
 * sources / targets as omap_maze_desc.  Validation of sizes and coordinates is
 * done here (same errors as omap_plan_create; a source on an obstacle is
 * reported FAILED at admission).  A query larger than the whole budget returns
 * OUT_OF_MEMORY.  *query_id receives a new id. */
omap_status_t omap_engine_submit(omap_engine_t engine, int32_t height, int32_t width,
                                 const uint8_t *occupancy_host,
                                 const int32_t *sources_host, int32_t n_sources,
                                 const int32_t *targets_host, int32_t n_targets,
                                 int64_t max_layers, int64_t *query_id);

/* omap_engine_submit with flags (0 or OMAP_QUERY_KEEP_ACTIVITY); same
 * validation and errors, plus INVALID_ARG for unknown flags. */
omap_status_t omap_engine_submit_ex(omap_engine_t engine, int32_t height, int32_t width,
                                    const uint8_t *occupancy_host,
                                    const int32_t *sources_host, int32_t n_sources,
                                    const int32_t *targets_host, int32_t n_targets,
                                    int64_t max_layers, uint32_t flags, int64_t *query_id);

/* One engine step: admit waiting queries that fit, advance all running
 * queries by `rounds` temporal blocks, and move converged queries through
 * retirement (paths, and kept activity maps, copied to host).  A query is
 * DONE a few steps after it converged.  *n_resident (queries holding a
 * slot) / *n_done_total (DONE or FAILED so far) may be NULL. */
omap_status_t omap_engine_step(omap_engine_t engine, int32_t rounds, int32_t *n_resident,
                               int64_t *n_done_total);

/* Ids of the queries that became DONE or FAILED since the previous call, in
 * the order they did: up to `capacity` of them go to ids_host (host) and
 * *n_ids receives their number; the others stay for the next call.  Host
 * only.  Errors: INVALID_ARG. */
omap_status_t omap_engine_completed(omap_engine_t engine, int64_t *ids_host, int32_t capacity, int32_t *n_ids);

/* State of a query: OMAP_QUERY_*.  NOT_FOUND for unknown / already fetched. */
omap_status_t omap_engine_poll(omap_engine_t engine, int64_t query_id, int32_t *state);

/* Fetch a finished query's results to host memory and forget it.
 *   len_host n_targets, offsets_host n_targets+1, cells_host cells_capacity;
 *   cells_needed_host always written; info_host may be NULL.
 * BUSY if not finished; BUFFER_TOO_SMALL leaves the query in place. */
omap_status_t omap_engine_fetch(omap_engine_t engine, int64_t query_id, int32_t *len_host,
                                int64_t *offsets_host, int32_t *cells_host,
                                int64_t cells_capacity, int64_t *cells_needed_host,
                                omap_propagate_info *info_host);

/* Activity map O of a DONE query submitted with OMAP_QUERY_KEEP_ACTIVITY
 * (the same map omap_get_activity gives for the maze alone):
 *   dst_host: height rows of width int32, row stride dst_pitch_elems >= width.
 * Call before omap_engine_fetch, which forgets the query.  Errors:
 * INVALID_ARG (NULL, pitch, flag not given), NOT_FOUND, BUSY. */
omap_status_t omap_engine_fetch_activity(omap_engine_t engine, int64_t query_id, int32_t *dst_host,
                                         int64_t dst_pitch_elems);

omap_status_t omap_engine_destroy(omap_engine_t engine);

/* ---------------------------------------------------------------------------
 * Autotuner: the tile shape and the layers per visit for a workload
 * ------------------------------------------------------------------------- */

#define OMAP_USE_PLAN 0     /* one maze per plan (n_mazes = 1)                    */
#define OMAP_USE_BATCH 1    /* many mazes advanced together                       */
#define OMAP_USE_ENGINE 2   /* a serving engine (the sample stands for its mix)   */

typedef struct omap_tune_result {
    omap_options options;   /* the fastest candidate: pass it to the create call  */
    int32_t candidates;     /* configurations timed (0 when read from the cache)  */
    int32_t from_cache;     /* 1 = options read from the OMAP_TUNE_CACHE file     */
    double best_ms;         /* propagation time of `options` on the sample        */
    double default_ms;      /* propagation time of the defaults on the sample     */
} omap_tune_result;

/* Picks options for a workload like `mazes` (device occupancy, as for
 * omap_batch_create): propagates the sample (run-time L) under the defaults
 * and under each candidate schedule / layers per visit / columns per lane /
 * tile rows, twice each (OMAP_USE_ENGINE: the sample propagated as one
 * batch stands for the engine's mix), keeps the fastest, and checks that
 * every candidate's
 * activity maps and layer counts equal the defaults' bit for bit (any tile
 * schedule reaches the same fixpoint; a difference fails the call with
 * OMAP_ERR_HIP).  With the environment variable OMAP_TUNE_CACHE naming a
 * file, choices are appended to it keyed by device, use, number of mazes and
 * median maze size (powers of two), and a later call for the same key reads
 * them back without timing anything.  Synchronous; needs device memory for
 * two copies of the sample's activity maps.  Errors: INVALID_ARG, those of
 * the create calls, OUT_OF_MEMORY, HIP. */
omap_status_t omap_tune(const omap_maze_desc *mazes, int32_t n_mazes, int32_t use,
                        omap_tune_result *result, void *stream);

/* ---------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------- */

/* Thread-local description of the last failure (never NULL). */
const char *omap_last_error(void);

/* Name of a status code (never NULL). */
const char *omap_status_string(omap_status_t status);

/* Kernel timing of a plan, batch or engine's tile-sweep kernel, collected with
 * HIP events on its stream while enabled (enable = 1 starts and clears,
 * enable = 0 stops).  *launches, *milliseconds, *cell_updates: totals since
 * enabling; cell_updates = interior cells of visited tiles x layers per visit.
 * kind: 0 plan, 1 batch, 2 engine. */
omap_status_t omap_profile_enable(void *handle, int32_t kind, int32_t enable);
omap_status_t omap_profile_read(void *handle, int32_t kind, int64_t *launches,
                                double *milliseconds, int64_t *cell_updates);

/* Runs the library's device self-checks (cross-lane moves and saturating
 * arithmetic the kernels rely on) on the current device.  Synchronous. */
omap_status_t omap_selftest(void *stream);

/* Library version string. */
const char *omap_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OMAP_H */
