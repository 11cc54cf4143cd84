// Host runtime of the oMAP planner: the multi-maze tile scheduler (Solver)
// behind the single-maze plan, the batch and the serving engine, and the C ABI
// declared in include/omap.h.
//
// All device work of a handle is ordered on one HIP stream.  A propagation is a
// sequence of rounds; one round is three launches: the tile sweep (T layers on
// every scheduled tile), the schedule build (next round's tile list from the
// change flags) and a per-maze update (counters, convergence).  The host reads
// the scheduled-tile count back only every few rounds, so the device never
// waits for a per-layer host handshake (the paper's appendix measures that
// handshake as the dominant cost of running one layer per call).

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unistd.h>
#include <unordered_map>
#include <vector>

#include "omap.h"
#include "omap_internal.h"

namespace omap {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error = "no error";

static omap_status_t fail(omap_status_t st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = std::string(omap_status_string(st)) + ": " + buf;
    return st;
}

omap_status_t report_error(omap_status_t st, const char* message) { return fail(st, "%s", message); }

// ---------------------------------------------------------------------------
// host copies
// ---------------------------------------------------------------------------

// Large host-to-host copies (a query's occupancy into pinned staging memory,
// a finished query's path cells out of it) split over a few worker threads:
// one core copies about 8 GB/s, which at tens of megabytes per query is the
// engine's largest host cost.  The workers are started on first use and live
// until the process ends; a copy returns when every chunk is done.
class CopyPool {
public:
    static CopyPool& get() {
        static CopyPool pool;
        return pool;
    }

    void copy(void* dst, const void* src, size_t n) {
        const size_t chunks = std::min<size_t>(workers_.size() + 1, n / kChunkMin);
        // (a process forked after the workers started has none of them)
        if (chunks < 2 || getpid() != pid_) {
            std::memcpy(dst, src, n);
            return;
        }
        Batch b;
        b.left = (int)chunks - 1;
        const size_t per = (n / chunks + 63) & ~size_t(63);
        {
            std::lock_guard<std::mutex> lk(m_);
            for (size_t k = 1; k < chunks; ++k) {
                const size_t off = k * per;
                if (off >= n) {
                    --b.left;
                    continue;
                }
                jobs_.push_back(Job{static_cast<char*>(dst) + off, static_cast<const char*>(src) + off,
                                    std::min(per, n - off), &b});
            }
        }
        cv_.notify_all();
        std::memcpy(dst, src, std::min(per, n));
        std::unique_lock<std::mutex> lk(m_);
        done_.wait(lk, [&] { return b.left == 0; });
    }

private:
    static constexpr size_t kChunkMin = size_t(1) << 20;
    struct Batch {
        int left = 0;
    };
    struct Job {
        char* dst;
        const char* src;
        size_t n;
        Batch* batch;
    };

    CopyPool() : pid_(getpid()) {
        const unsigned hw = std::thread::hardware_concurrency();
        const int n = (int)std::min(7u, hw > 2 ? hw / 2 : 0u);
        for (int i = 0; i < n; ++i) workers_.emplace_back([this] { run(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : workers_) t.join();
    }
    void run() {
        std::unique_lock<std::mutex> lk(m_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || !jobs_.empty(); });
            if (jobs_.empty()) return;   // stop_ with nothing left
            const Job j = jobs_.front();
            jobs_.pop_front();
            lk.unlock();
            std::memcpy(j.dst, j.src, j.n);
            lk.lock();
            if (--j.batch->left == 0) done_.notify_all();
        }
    }

    std::vector<std::thread> workers_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    std::deque<Job> jobs_;
    bool stop_ = false;
    const pid_t pid_;
};

static void host_copy(void* dst, const void* src, size_t n) { CopyPool::get().copy(dst, src, n); }

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return fail(_e == hipErrorOutOfMemory ? OMAP_ERR_OUT_OF_MEMORY : OMAP_ERR_HIP, \
                        "%s failed: %s", #expr, hipGetErrorString(_e));                 \
    } while (0)

#define OK_TRY(expr)                         \
    do {                                     \
        omap_status_t _s = (expr);           \
        if (_s != OMAP_OK) return _s;        \
    } while (0)

// ---------------------------------------------------------------------------
// options
// ---------------------------------------------------------------------------

struct Options {
    int T = 16;          // layers per tile visit
    int C = 4;           // columns per lane (strip = 64*C columns)
    int TH = 16;         // interior rows per tile
    int TW = 64 * 4 - 2 * 16;
    int dense = 0;
    int check = 0;       // 0 = adaptive
    int bits = 0;        // 1 = bit-sliced reached-set schedule (C unused; TW = 1984)
    int graph = 0;       // 1 = rounds replayed from captured HIP graphs
    int split = 0;       // 1 = two waves per tile visit (k_sweep_split: C = 1, T = TH = 16, active)
};

// Launch of one round's sweep kernel for the resolved options.
static hipError_t launch_round_kernel(const Options& opt, const RoundArgs& a, int32_t grid, hipStream_t s,
                                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    if (opt.bits) return launch_bits(opt.T, a, grid, s, e0, e1);
    if (opt.split) return launch_sweep_split_T16(a, grid, s, e0, e1);
    return launch_sweep(opt.T, opt.C, a, grid, s, e0, e1);
}

// Defaults (measured on MI355X).  A single maze under the active schedule is
// latency-bound (a few hundred tiles per round on 1024 SIMDs): one column per
// lane keeps each visit short, and with the one-column visits' unrolled
// warm-up 16 layers per visit beat 12 (23170^2 maze: propagation 8.2 vs
// 8.5 ms; 2 columns and 16 layers: 12.8 ms).  Many mazes at once (batch,
// engine) fill the device: there the bit-sliced schedule is fastest (512
// mazes: 19.6k mazes/s against 17.9k for the active schedule with 2 columns
// per lane and 12 layers per visit; serving capacity 198 against 180 mazes/s).
// The dense schedule is throughput-bound: 4 columns per lane, 16 layers and
// tall tiles.
enum class Use { kPlan, kMany };
static omap_status_t resolve_options(const omap_options* o, Options* out, Use use = Use::kPlan) {
    Options r;
    const bool single = use == Use::kPlan;
    int schedule = o ? o->schedule : OMAP_SCHEDULE_DEFAULT;
    if (schedule != OMAP_SCHEDULE_DEFAULT && schedule != OMAP_SCHEDULE_ACTIVE && schedule != OMAP_SCHEDULE_DENSE &&
        schedule != OMAP_SCHEDULE_BITS)
        return fail(OMAP_ERR_INVALID_ARG, "schedule must be DEFAULT, ACTIVE, DENSE or BITS (got %d)", schedule);
    if (schedule == OMAP_SCHEDULE_DEFAULT) {
        // the bit-sliced schedule has its own lane layout: an explicit column
        // count asks for the integer sweep
        schedule = (single || (o && o->lane_columns != 0)) ? OMAP_SCHEDULE_ACTIVE : OMAP_SCHEDULE_BITS;
        if (schedule == OMAP_SCHEDULE_BITS && o && o->temporal_depth != 0 && !bits_supported(o->temporal_depth))
            schedule = OMAP_SCHEDULE_ACTIVE;
    }
    const bool dense = schedule == OMAP_SCHEDULE_DENSE;
    const bool bits = schedule == OMAP_SCHEDULE_BITS;
    r.C = dense ? 4 : (single ? 1 : 2);
    r.T = 0;
    int th = 0;
    if (o) {
        if (o->lane_columns != 0) {
            if (o->lane_columns != 1 && o->lane_columns != 2 && o->lane_columns != 4)
                return fail(OMAP_ERR_INVALID_ARG, "lane_columns must be 1, 2 or 4 (got %d)", o->lane_columns);
            r.C = o->lane_columns;
        }
        r.T = o->temporal_depth;
        if (o->tile_rows != 0) {
            if (o->tile_rows < 2 || o->tile_rows > 4096 || (o->tile_rows & 1))
                return fail(OMAP_ERR_INVALID_ARG, "tile_rows must be even in [2, 4096] (got %d)",
                            o->tile_rows);
            th = o->tile_rows;
        }
        if (o->check_interval < 0) return fail(OMAP_ERR_INVALID_ARG, "check_interval < 0");
        r.check = o->check_interval;
        if (o->round_launch != OMAP_LAUNCH_PER_ROUND && o->round_launch != OMAP_LAUNCH_GRAPH)
            return fail(OMAP_ERR_INVALID_ARG, "round_launch must be PER_ROUND or GRAPH (got %d)", o->round_launch);
        r.graph = o->round_launch == OMAP_LAUNCH_GRAPH;
    }
    r.dense = dense;
    if (bits) {
        // bit-sliced: 32 columns per lane, one halo word per side
        if (o && o->lane_columns != 0)
            return fail(OMAP_ERR_INVALID_ARG, "lane_columns must be 0 with the bit-sliced schedule");
        r.bits = 1;
        r.C = 32;
        // many mazes: 8 layers per visit (the autotuner's choice on the 512-maze
        // batch, 21.4k against 19.6k mazes/s, and on the serving stream)
        if (r.T == 0) r.T = single ? 16 : 8;
        if (!bits_supported(r.T))
            return fail(OMAP_ERR_INVALID_ARG, "temporal_depth %d is not available with the bit-sliced schedule (8, 16)",
                        r.T);
        r.TH = th ? th : std::max(16, r.T);
        if (r.TH < r.T)
            return fail(OMAP_ERR_INVALID_ARG, "tile_rows (%d) must be >= temporal_depth (%d)", r.TH, r.T);
        r.TW = kBitsTileColumns;
        *out = r;
        return OMAP_OK;
    }
    if (r.T == 0) r.T = (dense || r.C == 1) ? 16 : 12;
    // a depth chosen without a column count takes the narrowest strip that has it
    if ((!o || o->lane_columns == 0) && !sweep_supported(r.T, r.C)) {
        if (sweep_supported(r.T, 2)) r.C = 2;
        else if (sweep_supported(r.T, 4)) r.C = 4;
    }
    if (!sweep_supported(r.T, r.C))
        return fail(OMAP_ERR_INVALID_ARG,
                    "temporal_depth %d is not available with %d columns per lane "
                    "(4, 8, 12, 16; with 2 columns also 24, 32)", r.T, r.C);
    // (with one column per lane the strip is 64 columns: 64 - 2T interior columns)
    r.TH = th ? th : (dense ? 256 : (single && r.C == 1 ? r.T : std::max(16, r.T)));
    if (r.TH < r.T)
        return fail(OMAP_ERR_INVALID_ARG, "tile_rows (%d) must be >= temporal_depth (%d)", r.TH, r.T);
    r.TW = 64 * r.C - 2 * r.T;
    // a single maze with one column per lane and 16 layers on 16-row tiles
    // (the latency-bound case) visits each tile with two waves
    r.split = single && !dense && r.C == 1 && r.T == 16 && r.TH == 16;
    *out = r;
    return OMAP_OK;
}

// ---------------------------------------------------------------------------
// device memory: direct allocation or a sub-allocated arena
// ---------------------------------------------------------------------------

class DeviceMemory {
   public:
    virtual ~DeviceMemory() {}
    virtual void* alloc(size_t bytes) = 0;   // nullptr on failure
    virtual void release(void* p) = 0;
};

class DirectMemory : public DeviceMemory {
   public:
    void* alloc(size_t bytes) override {
        void* p = nullptr;
        if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void release(void* p) override {
        if (p) (void)hipFree(p);
    }
};

// One allocation of the whole budget (device memory, or pinned host memory with
// `pinned`), carved into 256-byte aligned blocks by a best-fit free list.
// Reuse of device blocks after release is safe in stream order because all
// work of the owner runs on one stream; pinned blocks read by copies in flight
// are released through PinnedPool, which waits for those copies first.
class ArenaMemory : public DeviceMemory {
   public:
    ~ArenaMemory() override {
        if (base_) (void)(pinned_ ? hipHostFree(base_) : hipFree(base_));
    }
    void* base() const { return base_; }
    bool init(size_t bytes, bool pinned = false) {
        bytes = (bytes + 255) & ~size_t(255);
        pinned_ = pinned;
        const hipError_t e = pinned ? hipHostMalloc(&base_, bytes, hipHostMallocDefault) : hipMalloc(&base_, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            return false;
        }
        size_ = bytes;
        free_[0] = bytes;
        return true;
    }
    void* alloc(size_t bytes) override {
        bytes = (bytes + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return nullptr;
        const size_t off = best->first, len = best->second;
        free_.erase(best);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        in_use_ += bytes;
        return static_cast<char*>(base_) + off;
    }
    void release(void* p) override {
        if (!p) return;
        const size_t off = static_cast<char*>(p) - static_cast<char*>(base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t start = off, len = u->second;
        in_use_ -= len;
        used_.erase(u);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && nx->first == start + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
    }
    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    bool owns(const void* p) const {
        return base_ && p >= base_ && static_cast<const char*>(p) < static_cast<const char*>(base_) + size_;
    }

   private:
    void* base_ = nullptr;
    bool pinned_ = false;
    size_t size_ = 0, in_use_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> used_;
};

// Pinned host staging.  A host-to-device copy from pageable memory makes the
// host wait until the stream has drained up to it; staged through pinned
// memory it is a plain DMA in stream order, so the host can keep enqueueing
// work.  A block stays reserved until an event recorded after the copies that
// read it has completed.
class PinnedPool {
   public:
    ~PinnedPool() { clear(); }
    bool init(size_t bytes) { return arena_.init(bytes, true); }
    bool ready() const { return arena_.base() != nullptr; }
    size_t size() const { return arena_.size(); }

    // A pinned block of n bytes, nullptr if none is free even after waiting
    // for every pending release (the caller then copies from pageable memory).
    void* alloc(size_t n) {
        if (!ready() || n > arena_.size()) return nullptr;
        reap(false);
        void* p = arena_.alloc(n);
        while (!p && !pending_.empty()) {
            reap_one(true);
            p = arena_.alloc(n);
        }
        return p;
    }
    // Release p once the work enqueued on s so far has completed.
    hipError_t release_after(void* p, hipStream_t s) {
        hipEvent_t ev = nullptr;
        hipError_t e = spare_.empty() ? hipEventCreateWithFlags(&ev, hipEventDisableTiming) : hipSuccess;
        if (e != hipSuccess) return e;
        if (!ev) {
            ev = spare_.back();
            spare_.pop_back();
        }
        e = hipEventRecord(ev, s);
        if (e != hipSuccess) {
            spare_.push_back(ev);
            return e;
        }
        pending_.push_back({p, ev});
        return hipSuccess;
    }
    // Release p now (nothing in flight reads it).
    void release_now(void* p) { arena_.release(p); }
    bool owns(const void* p) const { return arena_.owns(p); }

    // Frees the blocks whose copies have completed (all of them with wait).
    void reap(bool wait) {
        while (!pending_.empty()) {
            if (!wait && hipEventQuery(pending_.front().second) != hipSuccess) {
                (void)hipGetLastError();
                break;
            }
            reap_one(true);
        }
    }

   private:
    void reap_one(bool wait) {
        auto [p, ev] = pending_.front();
        if (wait) (void)hipEventSynchronize(ev);
        pending_.pop_front();
        arena_.release(p);
        spare_.push_back(ev);
    }
    void clear() {
        for (auto& pe : pending_) {
            (void)hipEventSynchronize(pe.second);
            (void)hipEventDestroy(pe.second);
        }
        pending_.clear();
        for (hipEvent_t e : spare_) (void)hipEventDestroy(e);
        spare_.clear();
    }
    ArenaMemory arena_;
    std::deque<std::pair<void*, hipEvent_t>> pending_;
    std::vector<hipEvent_t> spare_;
};

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------

struct Geometry {
    int32_t H, W, pitch, mpitch, tiles_x, tiles_y;
    int64_t v_bytes, m_bytes;
    bool bits;                  // reached-set planes (m_bytes each) are needed
};

static Geometry make_geometry(int32_t H, int32_t W, const Options& o) {
    Geometry g;
    g.H = H;
    g.W = W;
    g.pitch = (W + 63) / 64 * 64;
    g.mpitch = g.pitch / 32;
    g.tiles_x = (W + o.TW - 1) / o.TW;
    g.tiles_y = (H + o.TH - 1) / o.TH;
    g.v_bytes = (int64_t)g.pitch * H * 4;
    g.m_bytes = (int64_t)g.mpitch * H * 4;
    g.bits = o.bits != 0;
    return g;
}

static int64_t maze_device_bytes(int32_t H, int32_t W, const Options& o) {
    const Geometry g = make_geometry(H, W, o);
    return 2 * g.v_bytes + (g.bits ? 3 : 1) * g.m_bytes + 4096;
}

static omap_status_t validate_problem(int32_t H, int32_t W, const void* occ,
                                      const int32_t* src, int32_t n_src, const int32_t* tgt,
                                      int32_t n_tgt) {
    if (H < 1 || W < 1) return fail(OMAP_ERR_INVALID_ARG, "height and width must be >= 1 (%d x %d)", H, W);
    if ((int64_t)H * W >= (int64_t(1) << 31))
        return fail(OMAP_ERR_TOO_LARGE, "height*width = %lld >= 2^31", (long long)H * W);
    if (!occ) return fail(OMAP_ERR_INVALID_ARG, "occupancy pointer is NULL");
    if (n_src < 1) return fail(OMAP_ERR_NO_SOURCES, "at least one source is required");
    if (!src) return fail(OMAP_ERR_INVALID_ARG, "sources pointer is NULL");
    if (n_tgt < 0) return fail(OMAP_ERR_INVALID_ARG, "n_targets < 0");
    if (n_tgt > 0 && !tgt) return fail(OMAP_ERR_INVALID_ARG, "targets pointer is NULL");
    for (int32_t i = 0; i < n_src; ++i)
        if (src[2 * i] < 0 || src[2 * i] >= H || src[2 * i + 1] < 0 || src[2 * i + 1] >= W)
            return fail(OMAP_ERR_SOURCE_OUT_OF_BOUNDS, "source %d at (%d, %d) outside %d x %d", i,
                        src[2 * i], src[2 * i + 1], H, W);
    for (int32_t i = 0; i < n_tgt; ++i)
        if (tgt[2 * i] < 0 || tgt[2 * i] >= H || tgt[2 * i + 1] < 0 || tgt[2 * i + 1] >= W)
            return fail(OMAP_ERR_TARGET_OUT_OF_BOUNDS, "target %d at (%d, %d) outside %d x %d", i,
                        tgt[2 * i], tgt[2 * i + 1], H, W);
    return OMAP_OK;
}

// ---------------------------------------------------------------------------
// Solver: resident mazes advanced together by tile rounds
// ---------------------------------------------------------------------------

struct Slot {
    bool used = false;
    Geometry g{};
    int32_t tile_base = 0, n_tiles = 0;
    int32_t* V[2] = {nullptr, nullptr};
    uint32_t* mask = nullptr;
    uint32_t* R[2] = {nullptr, nullptr};   // bit-sliced schedule only
    int32_t* d_src = nullptr;
    std::vector<int32_t> src, tgt;
    int32_t K = 0;
    int64_t L_req = 0;
    int64_t layers = -1;        // L or L* once finalized
    int64_t first_round = 0;    // round index of the maze's first visit
    int64_t reached = 0;
    bool started = false, finalized = false;
    bool cleared = false;       // both activity buffers are all zero outside touched tiles
};

class Solver {
   public:
    hipStream_t stream = nullptr;
    Options opt;
    DeviceMemory* mem = nullptr;
    int32_t cap_slots = 0, cap_tiles = 0;
    std::vector<Slot> slots;
    std::map<int32_t, int32_t> free_tiles;   // tile id range begin -> length
    int32_t tile_hwm = 0;                     // 1 + highest tile id ever handed out

    MazeDev* d_mazes = nullptr;
    int32_t* d_tile_maze = nullptr;
    int32_t* d_list[2] = {nullptr, nullptr};  // scheduled (tile id, slot) pairs by round mod 2
    int32_t* d_count = nullptr;               // [3] list counts by round mod 3
    int32_t* d_flags[2] = {nullptr, nullptr};
    int32_t* d_sched = nullptr;               // [3][cap_slots] scheduled tiles by round mod 3
    int32_t* d_dchg = nullptr;                // [3][cap_slots] dense: changed, by round mod 3
    int32_t* d_last_round = nullptr;          // per slot
    uint8_t* d_touched = nullptr;             // per tile id
    int64_t *d_visits = nullptr, *d_cell_visits = nullptr;
    unsigned long long* d_total_cells = nullptr;
    int32_t* d_bad_slot = nullptr;            // per slot: sources found on obstacles
    int32_t* h_bad = nullptr;                 // pinned mirror of d_bad_slot
    std::vector<MazeDev> h_mazes;             // host mirror of d_mazes
    std::vector<int32_t> h_tile_maze;         // host mirror of d_tile_maze
    int32_t* d_min = nullptr;
    unsigned long long* d_reached = nullptr;
    int32_t* d_bad = nullptr;
    int32_t* d_sel = nullptr;
    int32_t* h_pinned = nullptr;              // 64 int32 of pinned host scratch
    void* d_scratch = nullptr;                // grow-only path scratch
    size_t scratch_bytes = 0;
    int32_t* d_start_ = nullptr;              // grow-only staging of start_many
    size_t start_cap_ = 0;
    PinnedPool pin;                           // pinned staging of host-to-device copies

    int64_t next_round = 0;                   // index of the next round to run
    int parity = 0;                           // next_round mod 2: activity buffer holding the latest values
    int grid = 0;
    std::vector<void*> owned;                 // solver-level device allocations

    // profiling of the sweep kernel
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    std::vector<int64_t> prof_counts;         // launches each event pair brackets
    int64_t prof_launches = 0;
    double prof_ms = 0;
    unsigned long long prof_cells0 = 0;

    ~Solver() { destroy(); }

    void destroy() {
        for (auto& s : slots)
            if (s.used) free_slot_buffers(s);
        slots.clear();
        for (void* p : owned) (void)hipFree(p);
        owned.clear();
        if (d_scratch) (void)hipFree(d_scratch);
        d_scratch = nullptr;
        scratch_bytes = 0;
        if (d_start_) (void)hipFree(d_start_);
        d_start_ = nullptr;
        start_cap_ = 0;
        if (h_pinned) (void)hipHostFree(h_pinned);
        h_pinned = nullptr;
        if (h_bad) (void)hipHostFree(h_bad);
        h_bad = nullptr;
        if (h_fin_min) (void)hipHostFree(h_fin_min);
        h_fin_min = nullptr;
        if (h_fin_reached) (void)hipHostFree(h_fin_reached);
        h_fin_reached = nullptr;
        for (auto& e : prof_events) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        prof_events.clear();
        prof_counts.clear();
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
        gsig.clear();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        cap_stream = nullptr;
    }

    template <class Tp>
    omap_status_t dalloc(Tp** p, size_t n) {
        void* q = nullptr;
        HIP_TRY(hipMalloc(&q, n * sizeof(Tp) + 16));
        owned.push_back(q);
        *p = static_cast<Tp*>(q);
        return OMAP_OK;
    }

    // Stream-ordered host-to-device copy of n bytes that does not make the
    // host wait for the stream: staged through pinned memory when a block is
    // free, else copied from the caller's memory (then the host waits).
    omap_status_t upload(void* dst, const void* src, size_t n) {
        if (n == 0) return OMAP_OK;
        void* p = pin.alloc(n);
        if (p) {
            host_copy(p, src, n);
            HIP_TRY(hipMemcpyAsync(dst, p, n, hipMemcpyHostToDevice, stream));
            HIP_TRY(pin.release_after(p, stream));
            return OMAP_OK;
        }
        HIP_TRY(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return OMAP_OK;
    }

    omap_status_t init(hipStream_t s, const Options& o, DeviceMemory* m, int32_t slots_cap,
                       int32_t tiles_cap, size_t pinned_bytes = size_t(1) << 20) {
        stream = s;
        opt = o;
        mem = m;
        cap_slots = slots_cap;
        cap_tiles = tiles_cap;
        slots.assign(cap_slots, Slot());
        free_tiles.clear();
        free_tiles[0] = cap_tiles;
        OK_TRY(dalloc(&d_mazes, cap_slots));
        OK_TRY(dalloc(&d_tile_maze, cap_tiles));
        OK_TRY(dalloc(&d_list[0], 2 * (size_t)cap_tiles));   // (tile id, slot) pairs
        OK_TRY(dalloc(&d_list[1], 2 * (size_t)cap_tiles));
        OK_TRY(dalloc(&d_count, 3));
        OK_TRY(dalloc(&d_flags[0], cap_tiles));
        OK_TRY(dalloc(&d_flags[1], cap_tiles));
        OK_TRY(dalloc(&d_sched, 3 * (size_t)cap_slots));
        OK_TRY(dalloc(&d_dchg, 3 * (size_t)cap_slots));
        OK_TRY(dalloc(&d_last_round, cap_slots));
        OK_TRY(dalloc(&d_touched, cap_tiles));
        OK_TRY(dalloc(&d_bad_slot, cap_slots));
        HIP_TRY(hipHostMalloc((void**)&h_bad, sizeof(int32_t) * cap_slots, hipHostMallocDefault));
        h_mazes.assign(cap_slots, MazeDev());
        h_tile_maze.assign(cap_tiles, -1);
        OK_TRY(dalloc(&d_visits, (size_t)cap_slots * kSpread));
        OK_TRY(dalloc(&d_cell_visits, (size_t)cap_slots * kSpread));
        OK_TRY(dalloc(&d_total_cells, kSpread));
        OK_TRY(dalloc(&d_min, cap_slots));
        OK_TRY(dalloc(&d_reached, cap_slots));
        OK_TRY(dalloc(&d_bad, 1));
        OK_TRY(dalloc(&d_sel, cap_slots));
        HIP_TRY(hipHostMalloc((void**)&h_pinned, 64 * sizeof(int32_t), hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&h_fin_min, sizeof(int32_t) * cap_slots, hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&h_fin_reached, sizeof(unsigned long long) * cap_slots, hipHostMallocDefault));
        if (!pin.init(pinned_bytes)) return fail(OMAP_ERR_OUT_OF_MEMORY, "pinned staging (%zu bytes)", pinned_bytes);
        HIP_TRY(hipMemsetAsync(d_tile_maze, 0xff, sizeof(int32_t) * cap_tiles, stream));
        HIP_TRY(hipMemsetAsync(d_flags[0], 0, sizeof(int32_t) * cap_tiles, stream));
        HIP_TRY(hipMemsetAsync(d_flags[1], 0, sizeof(int32_t) * cap_tiles, stream));
        HIP_TRY(hipMemsetAsync(d_count, 0, 3 * sizeof(int32_t), stream));
        HIP_TRY(hipMemsetAsync(d_sched, 0, 3 * sizeof(int32_t) * cap_slots, stream));
        HIP_TRY(hipMemsetAsync(d_dchg, 0, 3 * sizeof(int32_t) * cap_slots, stream));
        HIP_TRY(hipMemsetAsync(d_last_round, 0, sizeof(int32_t) * cap_slots, stream));
        HIP_TRY(hipMemsetAsync(d_touched, 0, cap_tiles, stream));
        HIP_TRY(hipMemsetAsync(d_bad_slot, 0, sizeof(int32_t) * cap_slots, stream));
        HIP_TRY(hipMemsetAsync(d_visits, 0, sizeof(int64_t) * cap_slots * kSpread, stream));
        HIP_TRY(hipMemsetAsync(d_cell_visits, 0, sizeof(int64_t) * cap_slots * kSpread, stream));
        HIP_TRY(hipMemsetAsync(d_total_cells, 0, sizeof(unsigned long long) * kSpread, stream));
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        int cus = 0;
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        if (opt.split) {   // one tile per block of two waves
            grid = std::max(1, cus * std::max(1, sweep_split_blocks_per_cu_T16()));
            grid = std::max(1, std::min(grid, cap_tiles));
        } else {
            const int waves = opt.bits ? bits_max_waves_per_cu(opt.T) : sweep_max_waves_per_cu(opt.T, opt.C);
            grid = std::max(1, cus * std::max(1, waves / kWavesPerBlock));
            const int need = (cap_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
            grid = std::max(1, std::min(grid, need));
        }
        HIP_TRY(hipStreamSynchronize(stream));
        return OMAP_OK;
    }

    // Arguments of round r = next_round.  With `seeding` the "out" list,
    // count, flags and scheduled counts are those of round r itself (seeds
    // schedule tiles for the round about to run).
    RoundArgs round_args(bool seeding = false) const { return round_args_at(next_round, seeding); }

    RoundArgs round_args_at(int64_t r, bool seeding = false) const {
        RoundArgs a;
        std::memset(&a, 0, sizeof a);   // padding too: graph_signature compares the bytes
        const int r2 = (int)(r & 1), r3 = (int)(r % 3);
        const int n2 = r2 ^ 1, n3 = (r3 + 1) % 3, nn3 = (r3 + 2) % 3;
        a.mazes = d_mazes;
        a.tile_maze = d_tile_maze;
        a.n_tile_ids = tile_hwm;
        a.list_in = d_list[r2];
        a.count_in = d_count + r3;
        a.flags_in = d_flags[r2];
        a.list_out = d_list[seeding ? r2 : n2];
        a.count_out = d_count + (seeding ? r3 : n3);
        a.flags_out = d_flags[seeding ? r2 : n2];
        a.count_clear = d_count + nn3;
        a.sched_in = d_sched + (size_t)r3 * cap_slots;
        a.sched_out = d_sched + (size_t)(seeding ? r3 : n3) * cap_slots;
        a.sched_clear = d_sched + (size_t)nn3 * cap_slots;
        a.dchg_prev = d_dchg + (size_t)nn3 * cap_slots;   // written in round r-1
        a.dchg_cur = d_dchg + (size_t)r3 * cap_slots;
        a.dchg_clear = d_dchg + (size_t)n3 * cap_slots;
        a.maze_last_round = d_last_round;
        a.touched = d_touched;
        a.maze_visits = d_visits;
        a.maze_cell_visits = d_cell_visits;
        a.total_cells = d_total_cells;
        a.n_slots = cap_slots;
        a.round_id = (int32_t)r;
        a.round_base = nullptr;
        a.parity = r2;
        a.tile_rows = opt.TH;
        a.tile_cols = opt.TW;
        a.dense = opt.dense;
        a.md0 = h_mazes.empty() ? MazeDev() : h_mazes[0];
        return a;
    }

    void free_slot_buffers(Slot& s) {
        mem->release(s.V[0]);
        mem->release(s.V[1]);
        mem->release(s.mask);
        mem->release(s.d_src);
        if (s.R[0]) mem->release(s.R[0]);
        if (s.R[1]) mem->release(s.R[1]);
        s.V[0] = s.V[1] = nullptr;
        s.R[0] = s.R[1] = nullptr;
        s.mask = nullptr;
        s.d_src = nullptr;
    }

    // Copies slot k's descriptor to the device (stream-ordered; the host
    // mirror outlives the copy).
    omap_status_t upload_desc(int32_t k) {
        set_desc(k);
        return upload(d_mazes + k, &h_mazes[k], sizeof(MazeDev));
    }

    // Host mirror of slot k's descriptor.
    void set_desc(int32_t k) {
        const Slot& s = slots[k];
        MazeDev& md = h_mazes[k];
        md.H = s.g.H;
        md.W = s.g.W;
        md.pitch = s.g.pitch;
        md.mpitch = s.g.mpitch;
        md.tiles_x = s.g.tiles_x;
        md.tiles_y = s.g.tiles_y;
        md.tile_base = s.tile_base;
        md.K = s.K;
        md.V[0] = s.V[0];
        md.V[1] = s.V[1];
        md.mask = s.mask;
        md.R[0] = s.R[0];
        md.R[1] = s.R[1];
        md.round0 = (int32_t)s.first_round;
    }

    // Grow-only device staging of start_many (synchronizes only to grow; the
    // next start's upload is ordered after this start's kernels on the stream).
    omap_status_t start_scratch(size_t n_int32, int32_t** out) {
        if (n_int32 > start_cap_) {
            HIP_TRY(hipStreamSynchronize(stream));
            if (d_start_) (void)hipFree(d_start_);
            d_start_ = nullptr;
            start_cap_ = 0;
            const size_t want = std::max<size_t>(n_int32, 1024);
            HIP_TRY(hipMalloc(&d_start_, want * sizeof(int32_t)));
            start_cap_ = want;
        }
        *out = d_start_;
        return OMAP_OK;
    }

    omap_status_t upload_tile_range(int32_t base, int32_t n, int32_t value) {
        if (n <= 0) return OMAP_OK;
        std::fill(h_tile_maze.begin() + base, h_tile_maze.begin() + base + n, value);
        HIP_TRY(launch_fill(d_tile_maze + base, n, value, stream));
        return OMAP_OK;
    }

    bool take_tiles(int32_t n, int32_t* base) {
        for (auto it = free_tiles.begin(); it != free_tiles.end(); ++it) {
            if (it->second >= n) {
                *base = it->first;
                const int32_t rest = it->second - n, nb = it->first + n;
                free_tiles.erase(it);
                if (rest > 0) free_tiles[nb] = rest;
                tile_hwm = std::max(tile_hwm, *base + n);
                return true;
            }
        }
        return false;
    }

    void give_tiles(int32_t base, int32_t n) {
        auto nx = free_tiles.lower_bound(base);
        int32_t b = base, len = n;
        if (nx != free_tiles.end() && nx->first == b + len) {
            len += nx->second;
            nx = free_tiles.erase(nx);
        }
        if (nx != free_tiles.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == b) {
                b = pv->first;
                len += pv->second;
                free_tiles.erase(pv);
            }
        }
        free_tiles[b] = len;
    }

    int32_t free_slot_index() const {
        for (int32_t k = 0; k < cap_slots; ++k)
            if (!slots[k].used) return k;
        return -1;
    }

    // Pack one maze into slot k and check its sources on the device; the
    // verdict is read by commit() (stream-ordered, no host wait).
    // With check_sources = false the caller has checked the sources itself.
    omap_status_t pack_async(int32_t k, const uint8_t* occ_dev, const int32_t* src, int32_t n_src,
                             const int32_t* tgt, int32_t n_tgt, bool check_sources = true) {
        Slot& s = slots[k];
        OK_TRY(validate_problem(s.g.H, s.g.W, occ_dev, src, n_src, tgt, n_tgt));
        s.src.assign(src, src + 2 * n_src);
        if (tgt && n_tgt > 0) s.tgt.assign(tgt, tgt + 2 * n_tgt);
        else s.tgt.clear();
        HIP_TRY(launch_pack_mask(occ_dev, s.g.H, s.g.W, s.mask, s.g.mpitch, stream));
        if (check_sources) {
            mem->release(s.d_src);
            s.d_src = static_cast<int32_t*>(mem->alloc(sizeof(int32_t) * 2 * n_src));
            if (!s.d_src) return fail(OMAP_ERR_OUT_OF_MEMORY, "source list (%d sources)", n_src);
            OK_TRY(upload(s.d_src, s.src.data(), sizeof(int32_t) * 2 * n_src));
            HIP_TRY(launch_fill(d_bad_slot + k, 1, 0, stream));
            HIP_TRY(launch_check_sources(s.mask, s.g.mpitch, s.d_src, n_src, d_bad_slot + k, stream));
        }
        s.started = s.finalized = false;
        s.layers = -1;
        return OMAP_OK;
    }

    // Waits for the device and reports the first slot of `which` that has a
    // source on an obstacle (*bad_index = its position in `which`).
    omap_status_t commit(const std::vector<int32_t>& which, int32_t* bad_index) {
        HIP_TRY(hipMemcpyAsync(h_bad, d_bad_slot, sizeof(int32_t) * cap_slots, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        for (size_t i = 0; i < which.size(); ++i)
            if (h_bad[which[i]] != 0) {
                if (bad_index) *bad_index = (int32_t)i;
                return fail(OMAP_ERR_SOURCE_ON_OBSTACLE, "%d source(s) lie on obstacles", h_bad[which[i]]);
            }
        return OMAP_OK;
    }

    // Re-pack slot k with a new problem of the same size (synchronous).
    omap_status_t pack(int32_t k, const uint8_t* occ_dev, const int32_t* src, int32_t n_src,
                       const int32_t* tgt, int32_t n_tgt) {
        OK_TRY(pack_async(k, occ_dev, src, n_src, tgt, n_tgt));
        std::vector<int32_t> one{k};
        return commit(one, nullptr);
    }

    // Allocate slot buffers and a tile id range, then pack.  With defer the
    // source check is left to a later commit(); otherwise it is synchronous and
    // a failing maze is removed again.
    omap_status_t add(int32_t H, int32_t W, const uint8_t* occ_dev, const int32_t* src,
                      int32_t n_src, const int32_t* tgt, int32_t n_tgt, int32_t* slot_out,
                      bool defer = false, bool check_sources = true) {
        OK_TRY(validate_problem(H, W, occ_dev, src, n_src, tgt, n_tgt));
        const int32_t k = free_slot_index();
        if (k < 0) return fail(OMAP_ERR_OUT_OF_MEMORY, "no free maze slot (capacity %d)", cap_slots);
        Slot& s = slots[k];
        s = Slot();
        s.g = make_geometry(H, W, opt);
        const int64_t nt = (int64_t)s.g.tiles_x * s.g.tiles_y;
        if (nt > cap_tiles || !take_tiles((int32_t)nt, &s.tile_base))
            return fail(OMAP_ERR_OUT_OF_MEMORY, "no tile ids left for %lld tiles", (long long)nt);
        s.n_tiles = (int32_t)nt;
        s.used = true;
        s.V[0] = static_cast<int32_t*>(mem->alloc(s.g.v_bytes));
        s.V[1] = static_cast<int32_t*>(mem->alloc(s.g.v_bytes));
        s.mask = static_cast<uint32_t*>(mem->alloc(s.g.m_bytes));
        if (s.g.bits) {
            s.R[0] = static_cast<uint32_t*>(mem->alloc(s.g.m_bytes));
            s.R[1] = static_cast<uint32_t*>(mem->alloc(s.g.m_bytes));
        }
        if (!s.V[0] || !s.V[1] || !s.mask || (s.g.bits && (!s.R[0] || !s.R[1]))) {
            remove(k);
            return fail(OMAP_ERR_OUT_OF_MEMORY, "activity and mask buffers for %d x %d", H, W);
        }
        omap_status_t st = pack_async(k, occ_dev, src, n_src, tgt, n_tgt, check_sources);
        if (st == OMAP_OK) st = upload_tile_range(s.tile_base, s.n_tiles, k);
        if (st == OMAP_OK) st = upload_desc(k);
        if (st == OMAP_OK && !defer) {
            std::vector<int32_t> one{k};
            st = commit(one, nullptr);
        }
        if (st != OMAP_OK) {
            const std::string msg = g_last_error;
            remove(k);
            g_last_error = msg;
            return st;
        }
        *slot_out = k;
        return OMAP_OK;
    }

    // Add n mazes at once (batch creation): buffers and tile ids per maze on
    // the host side, then one copy each of the tile table, the descriptors and
    // the packing jobs and sources, one packing launch and one source check
    // for all of them.  The source verdicts are read by commit().
    omap_status_t add_many(const omap_maze_desc* d, int32_t n, std::vector<int32_t>* out_slots) {
        std::vector<PackJob> jobs;
        std::vector<int32_t> src_rc, src_slot;
        int64_t words = 0;
        for (int32_t i = 0; i < n; ++i) {
            OK_TRY(validate_problem(d[i].height, d[i].width, d[i].occupancy_dev, d[i].sources_host, d[i].n_sources,
                                    d[i].targets_host, d[i].n_targets));
            const int32_t k = free_slot_index();
            if (k < 0) return fail(OMAP_ERR_OUT_OF_MEMORY, "no free maze slot (capacity %d)", cap_slots);
            Slot& s = slots[k];
            s = Slot();
            s.g = make_geometry(d[i].height, d[i].width, opt);
            const int64_t nt = (int64_t)s.g.tiles_x * s.g.tiles_y;
            if (nt > cap_tiles || !take_tiles((int32_t)nt, &s.tile_base))
                return fail(OMAP_ERR_OUT_OF_MEMORY, "no tile ids left for %lld tiles", (long long)nt);
            s.n_tiles = (int32_t)nt;
            s.used = true;
            s.V[0] = static_cast<int32_t*>(mem->alloc(s.g.v_bytes));
            s.V[1] = static_cast<int32_t*>(mem->alloc(s.g.v_bytes));
            s.mask = static_cast<uint32_t*>(mem->alloc(s.g.m_bytes));
            if (s.g.bits) {
                s.R[0] = static_cast<uint32_t*>(mem->alloc(s.g.m_bytes));
                s.R[1] = static_cast<uint32_t*>(mem->alloc(s.g.m_bytes));
            }
            if (!s.V[0] || !s.V[1] || !s.mask || (s.g.bits && (!s.R[0] || !s.R[1])))
                return fail(OMAP_ERR_OUT_OF_MEMORY, "activity and mask buffers for %d x %d", d[i].height, d[i].width);
            s.src.assign(d[i].sources_host, d[i].sources_host + 2 * d[i].n_sources);
            if (d[i].targets_host && d[i].n_targets > 0)
                s.tgt.assign(d[i].targets_host, d[i].targets_host + 2 * d[i].n_targets);
            std::fill(h_tile_maze.begin() + s.tile_base, h_tile_maze.begin() + s.tile_base + s.n_tiles, k);
            PackJob jb;
            jb.occ = static_cast<const uint8_t*>(d[i].occupancy_dev);
            jb.mask = s.mask;
            jb.H = s.g.H;
            jb.W = s.g.W;
            jb.mpitch = s.g.mpitch;
            jb.word_begin = words;
            words += (int64_t)s.g.H * s.g.mpitch;
            jobs.push_back(jb);
            src_rc.insert(src_rc.end(), s.src.begin(), s.src.end());
            src_slot.insert(src_slot.end(), (size_t)d[i].n_sources, k);
            set_desc(k);
            out_slots->push_back(k);
        }
        const size_t b_jobs = (sizeof(PackJob) * jobs.size() + 255) & ~size_t(255);
        const size_t b_rc = (sizeof(int32_t) * src_rc.size() + 255) & ~size_t(255);
        const size_t b_sl = (sizeof(int32_t) * src_slot.size() + 255) & ~size_t(255);
        char* base = nullptr;
        OK_TRY(scratch(b_jobs + b_rc + b_sl, &base));
        std::vector<char> stage(b_jobs + b_rc + b_sl, 0);
        std::memcpy(stage.data(), jobs.data(), sizeof(PackJob) * jobs.size());
        std::memcpy(stage.data() + b_jobs, src_rc.data(), sizeof(int32_t) * src_rc.size());
        std::memcpy(stage.data() + b_jobs + b_rc, src_slot.data(), sizeof(int32_t) * src_slot.size());
        OK_TRY(upload(base, stage.data(), stage.size()));
        OK_TRY(upload(d_tile_maze, h_tile_maze.data(), sizeof(int32_t) * tile_hwm));
        OK_TRY(upload(d_mazes, h_mazes.data(), sizeof(MazeDev) * cap_slots));
        HIP_TRY(hipMemsetAsync(d_bad_slot, 0, sizeof(int32_t) * cap_slots, stream));
        HIP_TRY(launch_pack_mask_many(reinterpret_cast<const PackJob*>(base), n, words, stream));
        HIP_TRY(launch_check_sources_many(d_mazes, reinterpret_cast<const int32_t*>(base + b_jobs),
                                          reinterpret_cast<const int32_t*>(base + b_jobs + b_rc),
                                          (int32_t)src_slot.size(), d_bad_slot, stream));
        return OMAP_OK;
    }

    // Forget slot k: its tile ids and buffers go back to the pools
    // (stream-ordered).
    omap_status_t remove(int32_t k) {
        Slot& s = slots[k];
        if (!s.used) return OMAP_OK;
        if (s.n_tiles > 0) {
            OK_TRY(upload_tile_range(s.tile_base, s.n_tiles, -1));
            give_tiles(s.tile_base, s.n_tiles);
        }
        free_slot_buffers(s);
        s = Slot();
        return OMAP_OK;
    }

    // Reset slot k's activity and seed it for L layers (L < 0: run-time L).
    // Stream-ordered: the maze's tiles join the next round.
    omap_status_t start(int32_t k, int64_t L) {
        std::vector<int32_t> one{k};
        return start_many(one, &L);
    }

    // The same for several slots at once (Ls[i] for which[i]): one descriptor
    // copy, one clear, one reset and one seed launch for all of them.
    omap_status_t start_many(const std::vector<int32_t>& which, const int64_t* Ls) {
        if (which.empty()) return OMAP_OK;
        for (size_t i = 0; i < which.size(); ++i) {
            const int64_t L = Ls[i];
            if (L < -1) return fail(OMAP_ERR_INVALID_ARG, "max_layers must be >= 0 or OMAP_AUTO_LAYERS");
            if (L >= 0 && L + 1 > 0x7fffffffLL)
                return fail(OMAP_ERR_TOO_LARGE, "L + 1 = %lld does not fit int32 activity", (long long)(L + 1));
        }
        std::vector<int32_t> sel(cap_slots, 0), seed_slot;
        std::vector<int32_t> seed_rc;
        int32_t lo = tile_hwm, hi = 0;
        for (size_t i = 0; i < which.size(); ++i) {
            const int32_t k = which[i];
            Slot& s = slots[k];
            s.L_req = Ls[i];
            s.K = Ls[i] < 0 ? 0x7fffffff : (int32_t)(Ls[i] + 1);
            s.first_round = next_round;
            set_desc(k);
            sel[k] = 1;
            if (s.cleared) {
                lo = std::min(lo, s.tile_base);
                hi = std::max(hi, s.tile_base + s.n_tiles);
            }
            seed_rc.insert(seed_rc.end(), s.src.begin(), s.src.end());
            seed_slot.insert(seed_slot.end(), s.src.size() / 2, k);
        }
        OK_TRY(upload(d_mazes, h_mazes.data(), sizeof(MazeDev) * cap_slots));
        const RoundArgs a = round_args(true);
        // staging: selection | slot list | seed (r, c) pairs | seed slots
        const int32_t n_seed = (int32_t)seed_slot.size(), n_which = (int32_t)which.size();
        std::vector<int32_t> stage;
        stage.reserve(cap_slots + n_which + 3 * n_seed);
        stage.insert(stage.end(), sel.begin(), sel.end());
        stage.insert(stage.end(), which.begin(), which.end());
        stage.insert(stage.end(), seed_rc.begin(), seed_rc.end());
        stage.insert(stage.end(), seed_slot.begin(), seed_slot.end());
        int32_t* d_stage = nullptr;
        OK_TRY(start_scratch(stage.size(), &d_stage));
        OK_TRY(upload(d_stage, stage.data(), sizeof(int32_t) * stage.size()));
        const int32_t* d_sel_s = d_stage;
        const int32_t* d_which = d_stage + cap_slots;
        const int32_t* d_seed_rc = d_which + n_which;
        const int32_t* d_seed_slot = d_seed_rc + 2 * n_seed;
        if (hi > lo) HIP_TRY(launch_clear_touched(a, lo, hi - lo, d_sel_s, stream));
        for (int32_t k : which) {
            Slot& s = slots[k];
            if (s.cleared) continue;
            HIP_TRY(launch_fill(s.V[0], s.g.v_bytes / 4, 0, stream));
            HIP_TRY(launch_fill(s.V[1], s.g.v_bytes / 4, 0, stream));
            if (s.g.bits) {
                HIP_TRY(launch_fill(reinterpret_cast<int32_t*>(s.R[0]), s.g.m_bytes / 4, 0, stream));
                HIP_TRY(launch_fill(reinterpret_cast<int32_t*>(s.R[1]), s.g.m_bytes / 4, 0, stream));
            }
            HIP_TRY(hipMemsetAsync(d_touched + s.tile_base, 0, s.n_tiles, stream));
            s.cleared = true;
        }
        HIP_TRY(launch_slot_reset(a, d_which, n_which, stream));
        HIP_TRY(launch_seed(a, 0, d_seed_rc, d_seed_slot, n_seed, d_bad, stream));
        for (int32_t k : which) {
            Slot& s = slots[k];
            s.started = true;
            s.finalized = false;
            s.layers = -1;
        }
        return OMAP_OK;
    }

    // Empty schedule (before starting every resident maze afresh).
    omap_status_t reset_schedule() {
        HIP_TRY(hipMemsetAsync(d_count, 0, 3 * sizeof(int32_t), stream));
        HIP_TRY(hipMemsetAsync(d_flags[0], 0, sizeof(int32_t) * std::max(tile_hwm, 1), stream));
        HIP_TRY(hipMemsetAsync(d_flags[1], 0, sizeof(int32_t) * std::max(tile_hwm, 1), stream));
        HIP_TRY(hipMemsetAsync(d_sched, 0, 3 * sizeof(int32_t) * cap_slots, stream));
        HIP_TRY(hipMemsetAsync(d_dchg, 0, 3 * sizeof(int32_t) * cap_slots, stream));
        return OMAP_OK;
    }

    // One round: one sweep launch.
    omap_status_t round() {
        const RoundArgs a = round_args();
        if (prof) {
            std::pair<hipEvent_t, hipEvent_t> ev;
            // the events record the kernel's own start and end timestamps
            HIP_TRY(hipEventCreate(&ev.first));
            HIP_TRY(hipEventCreate(&ev.second));
            HIP_TRY(launch_round_kernel(opt, a, grid, stream, ev.first, ev.second));
            prof_events.push_back(ev);
            prof_counts.push_back(1);
        } else {
            HIP_TRY(launch_round_kernel(opt, a, grid, stream));
        }
        ++next_round;
        parity = (int)(next_round & 1);
        return OMAP_OK;
    }

    // ---- rounds replayed from a captured HIP graph (OMAP_LAUNCH_GRAPH) ----
    // A group of kGraphRounds round launches is captured once and replayed:
    // the round buffers rotate with period 6 (lists and flags by r mod 2,
    // counts by r mod 3), so a group that starts at a round r = 0 mod 6 has
    // the same arguments every time except the round numbers, which the
    // kernels take from a device counter (round_base) that a last node of the
    // group advances.  The graph is captured again whenever another argument
    // changes (a maze added or restarted, another tile id range).
    static constexpr int kGraphRounds = 24;
    hipStream_t cap_stream = nullptr;         // capture only (never runs work)
    hipGraphExec_t gexec = nullptr;
    std::vector<char> gsig;                   // arguments the graph was captured with
    int32_t* d_round_base = nullptr;

    std::vector<char> graph_signature() const {
        RoundArgs a = round_args_at(0);
        a.round_id = 0;
        std::vector<char> sig(sizeof(RoundArgs) + 3 * sizeof(int));
        std::memcpy(sig.data(), &a, sizeof a);
        const int extra[3] = {grid, opt.T, opt.C + 100 * opt.bits + 1000 * opt.split};
        std::memcpy(sig.data() + sizeof a, extra, sizeof extra);
        return sig;
    }

    omap_status_t graph_ensure() {
        std::vector<char> sig = graph_signature();
        if (gexec && sig == gsig) return OMAP_OK;
        if (gexec) (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
        gsig.clear();
        if (!d_round_base) OK_TRY(dalloc(&d_round_base, 1));
        if (!cap_stream) HIP_TRY(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed));
        hipError_t e = hipSuccess;
        for (int k = 0; k < kGraphRounds && e == hipSuccess; ++k) {
            RoundArgs a = round_args_at(k);
            a.round_id = k;
            a.round_base = d_round_base;
            e = launch_round_kernel(opt, a, grid, cap_stream);
        }
        if (e == hipSuccess) e = launch_round_advance(d_round_base, kGraphRounds, cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cap_stream, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            gexec = nullptr;
            return fail(OMAP_ERR_HIP, "capturing the round graph: %s", hipGetErrorString(e));
        }
        gsig.swap(sig);
        return OMAP_OK;
    }

    // At least `rounds` rounds: single launches up to the next multiple of 6,
    // then whole graph replays (the rest as single launches when
    // `exact`, else rounded up to whole replays).
    omap_status_t graph_rounds(int64_t rounds, bool exact) {
        int64_t done = 0;
        while (next_round % 6 != 0 && done < rounds) {
            OK_TRY(round());
            ++done;
        }
        int64_t reps = (rounds - done) / kGraphRounds;
        if (!exact && (rounds - done) % kGraphRounds != 0) ++reps;
        if (reps > 0) {
            OK_TRY(graph_ensure());
            HIP_TRY(launch_fill(d_round_base, 1, (int32_t)next_round, stream));
            std::pair<hipEvent_t, hipEvent_t> ev{};
            if (prof) {
                HIP_TRY(hipEventCreate(&ev.first));
                HIP_TRY(hipEventCreate(&ev.second));
                HIP_TRY(hipEventRecord(ev.first, stream));
            }
            for (int64_t i = 0; i < reps; ++i) HIP_TRY(hipGraphLaunch(gexec, stream));
            if (prof) {
                HIP_TRY(hipEventRecord(ev.second, stream));
                prof_events.push_back(ev);
                prof_counts.push_back(reps * kGraphRounds);
            }
            next_round += reps * kGraphRounds;
            done += reps * kGraphRounds;
            parity = (int)(next_round & 1);
        }
        while (done < rounds) {
            OK_TRY(round());
            ++done;
        }
        return OMAP_OK;
    }

    omap_status_t scheduled_count(int32_t* n) {
        HIP_TRY(hipMemcpyAsync(h_pinned, d_count + next_round % 3, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        *n = h_pinned[0];
        return OMAP_OK;
    }

    // Activity buffer holding the latest values: the round parity, except for
    // the bit-sliced schedule, which writes each reached cell's value once,
    // into buffer 0.
    int vparity() const { return opt.bits ? 0 : parity; }

    // `rounds` rounds.
    omap_status_t run_rounds(int32_t rounds) {
        if (opt.graph && rounds >= kGraphRounds + 5) return graph_rounds(rounds, true);
        for (int32_t i = 0; i < rounds; ++i) OK_TRY(round());
        return OMAP_OK;
    }

    // Rounds until no tile is scheduled (every started maze converged).
    omap_status_t run_to_convergence() {
        if (opt.graph) {
            // whole replays between count reads: 1, 2, 4, 4, ...
            int reps = 1;
            for (;;) {
                OK_TRY(graph_rounds((int64_t)reps * kGraphRounds, false));
                int32_t n = 0;
                OK_TRY(scheduled_count(&n));
                if (n == 0) return OMAP_OK;
                reps = std::min(reps * 2, 4);
            }
        }
        int g = opt.check > 0 ? opt.check : 2;
        for (;;) {
            for (int i = 0; i < g; ++i) OK_TRY(round());
            int32_t n = 0;
            OK_TRY(scheduled_count(&n));
            if (n == 0) break;
            if (opt.check == 0) g = std::min(g * 2, 64);
        }
        return OMAP_OK;
    }

    // Enqueues the reduction of the selected slots: their smallest positive
    // activity and reached count land in h_min / h_reached (pinned host
    // arrays of cap_slots entries) once the stream gets there.
    omap_status_t finalize_enqueue(const std::vector<int32_t>& which, int32_t* h_min, unsigned long long* h_reached) {
        HIP_TRY(launch_fill(d_min, cap_slots, 0x7fffffff, stream));
        HIP_TRY(launch_fill(reinterpret_cast<int32_t*>(d_reached), 2 * (int64_t)cap_slots, 0, stream));
        std::vector<int32_t> sel(cap_slots, 0);
        for (int32_t k : which) sel[k] = 1;
        OK_TRY(upload(d_sel, sel.data(), sizeof(int32_t) * cap_slots));
        int32_t lo = tile_hwm, hi = 0;
        for (int32_t k : which) {
            lo = std::min(lo, slots[k].tile_base);
            hi = std::max(hi, slots[k].tile_base + slots[k].n_tiles);
        }
        HIP_TRY(launch_reduce(d_mazes, d_tile_maze, d_touched, lo, hi, d_sel, opt.TH, opt.TW, vparity(), d_min,
                              d_reached, stream));
        HIP_TRY(hipMemcpyAsync(h_min, d_min, sizeof(int32_t) * cap_slots, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(h_reached, d_reached, sizeof(unsigned long long) * cap_slots, hipMemcpyDeviceToHost,
                               stream));
        return OMAP_OK;
    }

    // Layers (L or K - min) and reached counts of the selected slots from a
    // completed finalize_enqueue.
    void finalize_apply(const std::vector<int32_t>& which, const int32_t* h_min,
                        const unsigned long long* h_reached) {
        for (int32_t k : which) {
            Slot& s = slots[k];
            s.layers = s.L_req >= 0 ? s.L_req : (int64_t)s.K - h_min[k];
            s.reached = (int64_t)h_reached[k];
            s.finalized = true;
        }
    }

    // Pinned host arrays of the synchronous finalize (cap_slots each).
    int32_t* h_fin_min = nullptr;
    unsigned long long* h_fin_reached = nullptr;

    // Smallest positive activity and reached count of the selected slots,
    // then layers = L or K - min (synchronous).
    omap_status_t finalize(const std::vector<int32_t>& which) {
        OK_TRY(finalize_enqueue(which, h_fin_min, h_fin_reached));
        HIP_TRY(hipStreamSynchronize(stream));
        finalize_apply(which, h_fin_min, h_fin_reached);
        return OMAP_OK;
    }

    // Grow-only device scratch (synchronizes only when it has to grow).
    omap_status_t scratch(size_t bytes, char** out) {
        if (bytes > scratch_bytes) {
            HIP_TRY(hipStreamSynchronize(stream));
            if (d_scratch) (void)hipFree(d_scratch);
            d_scratch = nullptr;
            scratch_bytes = 0;
            const size_t want = std::max(bytes, scratch_bytes * 2);
            HIP_TRY(hipMalloc(&d_scratch, want));
            scratch_bytes = want;
        }
        *out = static_cast<char*>(d_scratch);
        return OMAP_OK;
    }

    omap_status_t ensure_finalized(int32_t k) {
        if (slots[k].finalized) return OMAP_OK;
        std::vector<int32_t> one{k};
        return finalize(one);
    }

    // Host copies of every slot's visit counters (read_counters, synchronous).
    std::vector<int32_t> h_last_round;
    std::vector<int64_t> h_visits, h_cell_visits;

    omap_status_t read_counters() {
        h_last_round.resize(cap_slots);
        h_visits.resize((size_t)cap_slots * kSpread);
        h_cell_visits.resize((size_t)cap_slots * kSpread);
        HIP_TRY(hipMemcpyAsync(h_last_round.data(), d_last_round, sizeof(int32_t) * cap_slots, hipMemcpyDeviceToHost,
                               stream));
        HIP_TRY(hipMemcpyAsync(h_visits.data(), d_visits, sizeof(int64_t) * h_visits.size(), hipMemcpyDeviceToHost,
                               stream));
        HIP_TRY(hipMemcpyAsync(h_cell_visits.data(), d_cell_visits, sizeof(int64_t) * h_cell_visits.size(),
                               hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return OMAP_OK;
    }

    // Report of slot k; with counters_read the host copies of read_counters()
    // are used instead of reading the device.
    omap_status_t info(int32_t k, omap_propagate_info* out, bool counters_read = false) {
        OK_TRY(ensure_finalized(k));
        if (!counters_read) {
            OK_TRY(read_counters());
        }
        int64_t v[3] = {0, 0, 0};
        for (int j = 0; j < kSpread; ++j) {
            v[1] += h_visits[(size_t)k * kSpread + j];
            v[2] += h_cell_visits[(size_t)k * kSpread + j];
        }
        const Slot& s = slots[k];
        v[0] = (int64_t)(int32_t)(h_last_round[k] - (int32_t)s.first_round) + 1;   // rounds the maze was visited
        if (v[0] < 0) v[0] = 0;
        out->layers = s.layers;
        out->rounds = v[0];
        out->sweeps_executed = v[0] * opt.T;
        out->tile_visits = v[1];
        out->reached_cells = s.reached;
        return OMAP_OK;
    }

    // Paths of the targets of `which` (in that order), written to caller
    // buffers: device buffers, or host buffers with host_out.  mode: 0 simple
    // reconstruction (fixed tie order), 1 simple with seeded random ties,
    // 2 Euclidean.  src_out (optional): index of the source each path ends on.
    // Scratch comes from a grow-only device buffer.
    omap_status_t extract(const std::vector<int32_t>& which, int32_t* len_out, int64_t* off_out,
                          int32_t* cells_out, int64_t capacity, int64_t* needed, bool host_out,
                          int mode = 0, uint64_t seed = 0, int32_t* src_out = nullptr) {
        std::vector<int32_t> tslot, trc, tlocal, sbase, scount, ssorted;
        for (int32_t k : which) {
            const Slot& s = slots[k];
            if (!s.started) return fail(OMAP_ERR_NOT_PROPAGATED, "maze %d has not been propagated", k);
            const int32_t n = (int32_t)(s.tgt.size() / 2);
            tslot.insert(tslot.end(), n, k);
            trc.insert(trc.end(), s.tgt.begin(), s.tgt.end());
            for (int32_t t = 0; t < n; ++t) tlocal.push_back(t);
            if (src_out) {
                // (linear cell, first list index), sorted by cell, duplicates dropped
                std::vector<std::pair<int32_t, int32_t>> v;
                for (size_t j = 0; j < s.src.size() / 2; ++j)
                    v.push_back({s.src[2 * j] * s.g.W + s.src[2 * j + 1], (int32_t)j});
                std::sort(v.begin(), v.end());
                v.erase(std::unique(v.begin(), v.end(),
                                    [](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
                                        return a.first == b.first;
                                    }),
                        v.end());
                const int32_t base = (int32_t)(ssorted.size() / 2);
                for (auto& e : v) {
                    ssorted.push_back(e.first);
                    ssorted.push_back(e.second);
                }
                sbase.insert(sbase.end(), n, base);
                scount.insert(scount.end(), n, (int32_t)v.size());
            }
        }
        const int32_t n = (int32_t)tslot.size();
        auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
        const size_t b_i = up(sizeof(int32_t) * (n + 1)), b_rc = up(sizeof(int32_t) * (2 * n + 2));
        const size_t b_off = up(sizeof(int64_t) * (n + 1)), b_ss = up(sizeof(int32_t) * (ssorted.size() + 2));
        // layout: tslot | trc | tlocal | len | off | sbase | scount | ssorted | order | (cells for host_out)
        const size_t fixed = b_i + b_rc + b_i + b_i + b_off + b_i + b_i + b_ss + b_i;
        char* base = nullptr;
        OK_TRY(scratch(fixed, &base));
        auto carve = [&](char* b) {
            struct P { int32_t *tslot, *trc, *tlocal, *len; int64_t* off; int32_t *sbase, *scount, *ss, *order; char* end; } q;
            q.tslot = reinterpret_cast<int32_t*>(b); b += b_i;
            q.trc = reinterpret_cast<int32_t*>(b); b += b_rc;
            q.tlocal = reinterpret_cast<int32_t*>(b); b += b_i;
            q.len = reinterpret_cast<int32_t*>(b); b += b_i;
            q.off = reinterpret_cast<int64_t*>(b); b += b_off;
            q.sbase = reinterpret_cast<int32_t*>(b); b += b_i;
            q.scount = reinterpret_cast<int32_t*>(b); b += b_i;
            q.ss = reinterpret_cast<int32_t*>(b); b += b_ss;
            q.order = reinterpret_cast<int32_t*>(b); b += b_i;
            q.end = b;
            return q;
        };
        auto q = carve(base);
        // lengths and offsets (the Euclidean walk learns its lengths by walking)
        auto lengths = [&](decltype(q)& d) -> omap_status_t {
            if (n > 0) {
                OK_TRY(upload(d.tslot, tslot.data(), sizeof(int32_t) * n));
                OK_TRY(upload(d.trc, trc.data(), sizeof(int32_t) * 2 * n));
                OK_TRY(upload(d.tlocal, tlocal.data(), sizeof(int32_t) * n));
                if (src_out) {
                    OK_TRY(upload(d.sbase, sbase.data(), sizeof(int32_t) * n));
                    OK_TRY(upload(d.scount, scount.data(), sizeof(int32_t) * n));
                    OK_TRY(upload(d.ss, ssorted.data(), sizeof(int32_t) * ssorted.size()));
                }
                if (mode == 2)
                    HIP_TRY(launch_walk_euclid(false, d_mazes, d.tslot, d.trc, n, vparity(), d.len, nullptr, nullptr, stream));
                else
                    HIP_TRY(launch_path_lengths(d_mazes, d.tslot, d.trc, n, vparity(), d.len, stream));
            }
            HIP_TRY(launch_scan_offsets(d.len, n, d.off, stream, mode == 0 ? d.order : nullptr));
            return OMAP_OK;
        };
        OK_TRY(lengths(q));
        HIP_TRY(hipMemcpyAsync(h_pinned, q.off + n, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        int64_t total = 0;
        std::memcpy(&total, h_pinned, sizeof total);
        if (needed) *needed = total;
        if (capacity < total || (total > 0 && cells_out == nullptr))
            return fail(OMAP_ERR_BUFFER_TOO_SMALL, "paths need %lld cells, capacity %lld",
                        (long long)total, (long long)capacity);
        int32_t* walk_dst = cells_out;
        if (host_out || src_out) {
            // cells go to scratch first (host copy and/or source lookup read them there)
            const size_t b_cells = up(sizeof(int32_t) * (size_t)(total + 1));
            char* base2 = nullptr;
            OK_TRY(scratch(fixed + b_cells, &base2));
            if (base2 != base) {   // scratch moved: redo the lengths in the new place
                q = carve(base2);
                OK_TRY(lengths(q));
                base = base2;
            }
            if (host_out) walk_dst = reinterpret_cast<int32_t*>(q.end);
        }
        if (mode == 2)
            HIP_TRY(launch_walk_euclid(true, d_mazes, q.tslot, q.trc, n, vparity(), q.len, q.off, walk_dst, stream));
        else if (mode == 1)
            HIP_TRY(launch_walk_random(d_mazes, q.tslot, q.trc, q.tlocal, n, vparity(), seed, q.len, q.off, walk_dst, stream));
        else
            HIP_TRY(launch_walk(d_mazes, q.tslot, q.trc, n, vparity(), q.len, q.off, walk_dst, stream, q.order));
        const hipMemcpyKind kind = host_out ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
        if (src_out)
            HIP_TRY(launch_source_index(d_mazes, q.tslot, n, q.len, q.off, walk_dst, q.ss, q.sbase, q.scount,
                                        src_out, stream));
        if (n > 0) HIP_TRY(hipMemcpyAsync(len_out, q.len, sizeof(int32_t) * n, kind, stream));
        HIP_TRY(hipMemcpyAsync(off_out, q.off, sizeof(int64_t) * (n + 1), kind, stream));
        if (host_out && total > 0)
            HIP_TRY(hipMemcpyAsync(cells_out, walk_dst, sizeof(int32_t) * total, kind, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return OMAP_OK;
    }

    omap_status_t activity(int32_t k, int32_t* dst, int64_t dpitch) {
        Slot& s = slots[k];
        if (!dst) return fail(OMAP_ERR_INVALID_ARG, "destination is NULL");
        if (dpitch < s.g.W) return fail(OMAP_ERR_INVALID_ARG, "pitch %lld < width %d", (long long)dpitch, s.g.W);
        if (!s.started) return fail(OMAP_ERR_NOT_PROPAGATED, "maze %d has not been propagated", k);
        OK_TRY(ensure_finalized(k));
        const int64_t off = (int64_t)s.K - s.layers - 1;
        HIP_TRY(launch_activity(d_mazes, k, s.g.H, s.g.W, vparity(), (int32_t)off, dst, dpitch, stream));
        return OMAP_OK;
    }

    // Sum of the visit-cell counter copies (synchronous).
    omap_status_t total_cells(unsigned long long* out) {
        unsigned long long c[kSpread];
        HIP_TRY(hipMemcpyAsync(c, d_total_cells, sizeof c, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        *out = 0;
        for (int j = 0; j < kSpread; ++j) *out += c[j];
        return OMAP_OK;
    }

    omap_status_t profile(bool on) {
        if (on) {
            for (auto& e : prof_events) {
                (void)hipEventDestroy(e.first);
                (void)hipEventDestroy(e.second);
            }
            prof_events.clear();
            prof_counts.clear();
            prof_launches = 0;
            prof_ms = 0;
            OK_TRY(total_cells(&prof_cells0));
        }
        prof = on;
        return OMAP_OK;
    }

    omap_status_t profile_read(int64_t* launches, double* ms, int64_t* cell_updates) {
        HIP_TRY(hipStreamSynchronize(stream));
        for (size_t i = 0; i < prof_events.size(); ++i) {
            auto& e = prof_events[i];
            float t = 0;
            HIP_TRY(hipEventElapsedTime(&t, e.first, e.second));
            prof_ms += t;
            prof_launches += prof_counts[i];
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        prof_events.clear();
        prof_counts.clear();
        unsigned long long cells = 0;
        OK_TRY(total_cells(&cells));
        if (launches) *launches = prof_launches;
        if (ms) *ms = prof_ms;
        if (cell_updates) *cell_updates = (int64_t)(cells - prof_cells0) * opt.T;
        return OMAP_OK;
    }
};

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------

}  // namespace omap

struct omap_plan_s {
    omap::DirectMemory mem;
    omap::Solver solver;
    int32_t slot = -1;
    int device = 0;          // device current at create
    bool propagated = false;
};

struct omap_batch_s {
    omap::ArenaMemory mem;   // one device allocation holding every maze's buffers
    omap::Solver solver;
    std::vector<int32_t> slots;
    bool propagated = false;
};

namespace omap {

struct Query {
    int64_t id = 0;
    int32_t H = 0, W = 0;
    std::vector<uint8_t> occ;     // copy of the occupancy when no pinned block was free at submit
    uint8_t* occ_pinned = nullptr;
    std::vector<int32_t> src, tgt;
    int64_t L = -1;
    uint32_t flags = 0;           // OMAP_QUERY_KEEP_ACTIVITY
    int32_t state = OMAP_QUERY_QUEUED;
    int32_t slot = -1;
    int64_t bytes = 0;
    std::string error;
    std::vector<int32_t> len;
    std::vector<int64_t> off;
    std::vector<int32_t> cells;
    int32_t* cells_pinned = nullptr; // the path cells in the engine's pinned result pool (else in `cells`)
    int64_t n_cells = 0;
    std::vector<int32_t> activity;   // kept activity map (H x W) with OMAP_QUERY_KEEP_ACTIVITY
    omap_propagate_info info{};
};

// Grow-only pinned host buffer.
struct PinnedBuffer {
    char* p = nullptr;
    size_t size = 0;
    ~PinnedBuffer() {
        if (p) (void)hipHostFree(p);
    }
    omap_status_t reserve(size_t bytes) {
        if (bytes <= size) return OMAP_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        size = 0;
        const size_t want = std::max(bytes, size_t(1) << 20);
        HIP_TRY(hipHostMalloc((void**)&p, want, hipHostMallocDefault));
        size = want;
        return OMAP_OK;
    }
};

// Per-slot convergence counts copied to the host after a step's rounds.
struct Snapshot {
    int32_t* counts = nullptr;   // pinned, cap_slots entries
    hipEvent_t ev = nullptr;
    int64_t round = 0;           // next_round when the copy was enqueued
    bool busy = false;
};

// Retirement of the mazes found converged together, in three stream-ordered
// phases so that the host never waits for the device: (1) finalize and path
// lengths, (2) once their sizes are known on the host, the walk and the copies
// of paths, counters and kept activity maps, (3) the results handed to the
// queries and the slots freed.
struct Retirement {
    int phase = 0;               // 0 idle, 1 lengths in flight, 2 paths in flight
    std::vector<int64_t> ids;
    std::vector<int32_t> slots;
    int32_t n = 0;               // targets of all of them
    int64_t total = 0;           // path cells of all of them
    hipEvent_t ev = nullptr;
    int32_t* h_min = nullptr;    // pinned, cap_slots
    unsigned long long* h_reached = nullptr;
    PinnedBuffer h_lo;           // lengths, offsets
    PinnedBuffer h_out;          // counters, cells, kept activity maps
    std::vector<int64_t> act_off;   // per retiring query: byte offset of its map in h_out (-1 = none)
    std::vector<void*> cells_block; // per retiring query: its cells' block of the result pool (or null)
    int32_t* d_cells = nullptr;  // grow-only device buffers
    size_t cells_cap = 0;
    int32_t* d_act = nullptr;
    size_t act_cap = 0;
};

}  // namespace omap

struct omap_engine_s {
    omap::ArenaMemory mem;
    omap::Solver solver;
    omap::PinnedPool occ_pool;       // pinned copies of submitted occupancy grids
    omap::PinnedPool res_pool;       // pinned path cells of finished queries until fetched
    // Second stream (default priority) for what need not wait for the rounds:
    // occupancy uploads of the next admissions and the walks and copies of a
    // retirement.  The rounds stay on the solver's stream.
    hipStream_t xfer = nullptr;
    struct Staged {
        int64_t id;
        void* occ_dev;               // occupancy on the device (arena), uploaded on xfer
        hipEvent_t ev;               // the upload's completion
        int64_t reserve;             // bytes reserved for the maze's buffers
    };
    std::deque<Staged> staged;       // uploaded or uploading, admitted at a later step
    int64_t reserved = 0;
    std::deque<std::pair<void*, hipEvent_t>> dev_release;   // arena blocks freed once the event completes
    std::vector<hipEvent_t> ev_spare;
    std::deque<int64_t> completed;   // DONE / FAILED ids not yet handed out by omap_engine_completed
    int64_t budget = 0;
    int32_t max_slots = 0;
    int64_t next_id = 1;
    int64_t done_total = 0;
    std::deque<int64_t> waiting;
    std::unordered_map<int64_t, omap::Query> queries;
    std::vector<int64_t> running;     // admitted, not yet seen converged
    std::vector<int64_t> converged;   // seen converged, waiting for a retirement
    omap::Snapshot snap[2];
    int snap_next = 0;                // snapshot slot the next copy goes to
    omap::Retirement ret;

    ~omap_engine_s() {
        (void)hipStreamSynchronize(solver.stream);
        if (xfer) (void)hipStreamSynchronize(xfer);
        for (auto& st : staged) (void)hipEventDestroy(st.ev);
        for (auto& r : dev_release) (void)hipEventDestroy(r.second);
        for (hipEvent_t ev : ev_spare) (void)hipEventDestroy(ev);
        if (xfer) (void)hipStreamDestroy(xfer);
        for (auto& sn : snap) {
            if (sn.ev) (void)hipEventDestroy(sn.ev);
            if (sn.counts) (void)hipHostFree(sn.counts);
        }
        if (ret.ev) (void)hipEventDestroy(ret.ev);
        if (ret.h_min) (void)hipHostFree(ret.h_min);
        if (ret.h_reached) (void)hipHostFree(ret.h_reached);
        if (ret.d_cells) (void)hipFree(ret.d_cells);
        if (ret.d_act) (void)hipFree(ret.d_act);
    }
    int32_t resident() const {
        return (int32_t)(staged.size() + running.size() + converged.size() + ret.ids.size());
    }
    hipError_t event(hipEvent_t* ev) {
        if (!ev_spare.empty()) {
            *ev = ev_spare.back();
            ev_spare.pop_back();
            return hipSuccess;
        }
        return hipEventCreateWithFlags(ev, hipEventDisableTiming);
    }
};

namespace omap {

// Byte offset of the offsets array in a retirement's lengths / offsets buffer.
static size_t lo_offsets_at(size_t n) { return (4 * (n + 1) + 63) & ~size_t(63); }

static int64_t query_bytes(const Query& q, const Options& o) {
    // activity ping-pong + mask + staging of the occupancy + path scratch
    const int64_t nt = (int64_t)q.tgt.size() / 2;
    return maze_device_bytes(q.H, q.W, o) + (int64_t)q.H * q.W + 256 +
           nt * 64 + nt * 4 * ((int64_t)q.H + q.W) + 4096;
}

static void query_release_occ(omap_engine_s* e, Query& q) {
    if (q.occ_pinned) e->occ_pool.release_now(q.occ_pinned);
    q.occ_pinned = nullptr;
    q.occ.clear();
    q.occ.shrink_to_fit();
}

static void query_fail(omap_engine_s* e, Query& q, const std::string& msg) {
    q.state = OMAP_QUERY_FAILED;
    q.error = msg;
    q.slot = -1;
    query_release_occ(e, q);
    ++e->done_total;
    e->completed.push_back(q.id);
}

// Arena blocks whose last reader has completed go back to the arena.
static void engine_reap(omap_engine_s* e) {
    while (!e->dev_release.empty()) {
        const hipError_t r = hipEventQuery(e->dev_release.front().second);
        if (r == hipErrorNotReady) {
            (void)hipGetLastError();
            break;
        }
        e->mem.release(e->dev_release.front().first);
        e->ev_spare.push_back(e->dev_release.front().second);
        e->dev_release.pop_front();
    }
    e->occ_pool.reap(false);
}

// Admission in two steps so that no upload holds up the rounds.  Staged
// queries whose occupancy has arrived are packed and started together on the
// solver's stream; then waiting queries that fit (a slot, and device memory
// for the occupancy plus a reservation for the maze's buffers) are staged:
// sources checked on the host copy, occupancy copied to the device on the
// transfer stream.  Nothing here waits for the device.
static omap_status_t engine_admit(omap_engine_s* e) {
    Solver& sv = e->solver;
    engine_reap(e);
    std::vector<int32_t> started;
    std::vector<int64_t> Ls, ids;
    while (!e->staged.empty()) {
        omap_engine_s::Staged& g = e->staged.front();
        const hipError_t r = hipEventQuery(g.ev);
        if (r == hipErrorNotReady) {
            (void)hipGetLastError();
            break;   // the uploads complete in order
        }
        Query& q = e->queries[g.id];
        e->reserved -= g.reserve;
        int32_t slot = -1;
        omap_status_t st = r == hipSuccess
                               ? sv.add(q.H, q.W, static_cast<uint8_t*>(g.occ_dev), q.src.data(),
                                        (int32_t)(q.src.size() / 2), q.tgt.empty() ? nullptr : q.tgt.data(),
                                        (int32_t)(q.tgt.size() / 2), &slot, /*defer=*/true, /*check_sources=*/false)
                               : fail(OMAP_ERR_HIP, "occupancy upload: %s", hipGetErrorString(r));
        if (st == OMAP_ERR_OUT_OF_MEMORY && e->resident() > (int32_t)e->staged.size()) {
            e->reserved += g.reserve;   // fragmented arena: retry when something retires
            break;
        }
        // the staging block is read by the packing kernel: freed once that has run
        hipEvent_t done = g.ev;
        HIP_TRY(hipEventRecord(done, sv.stream));
        e->dev_release.push_back({g.occ_dev, done});
        const int64_t id = g.id;
        e->staged.pop_front();
        if (st != OMAP_OK) {
            query_fail(e, e->queries[id], g_last_error);
            continue;
        }
        e->queries[id].slot = slot;
        started.push_back(slot);
        Ls.push_back(e->queries[id].L);
        ids.push_back(id);
    }
    if (!started.empty()) {
        omap_status_t st = sv.start_many(started, Ls.data());
        if (st != OMAP_OK) {
            const std::string msg = g_last_error;
            for (size_t i = 0; i < ids.size(); ++i) {
                sv.remove(started[i]);
                query_fail(e, e->queries[ids[i]], msg);
            }
            g_last_error = msg;
        } else {
            for (int64_t id : ids) {
                e->queries[id].state = OMAP_QUERY_RUNNING;
                e->running.push_back(id);
            }
        }
    }
    while (!e->waiting.empty() && e->resident() < e->max_slots) {
        Query& q = e->queries[e->waiting.front()];
        if ((int64_t)e->mem.in_use() + e->reserved + q.bytes > (int64_t)e->mem.size()) break;   // wait for memory
        const uint8_t* occ_host = q.occ_pinned ? q.occ_pinned : q.occ.data();
        int32_t bad = 0;
        for (size_t j = 0; j < q.src.size(); j += 2)
            bad += occ_host[(int64_t)q.src[j] * q.W + q.src[j + 1]] != 0;
        if (bad) {
            e->waiting.pop_front();
            query_fail(e, q, std::string(omap_status_string(OMAP_ERR_SOURCE_ON_OBSTACLE)) + ": " +
                                 std::to_string(bad) + " source(s) lie on obstacles");
            continue;
        }
        const size_t n_occ = (size_t)q.H * q.W;
        void* occ_dev = e->mem.alloc(n_occ);
        if (!occ_dev) break;
        omap_engine_s::Staged g{q.id, occ_dev, nullptr, std::max<int64_t>(0, q.bytes - (int64_t)n_occ)};
        hipError_t r = e->event(&g.ev);
        if (r == hipSuccess) {
            if (q.occ_pinned) {
                r = hipMemcpyAsync(occ_dev, q.occ_pinned, n_occ, hipMemcpyHostToDevice, e->xfer);
                if (r == hipSuccess) r = e->occ_pool.release_after(q.occ_pinned, e->xfer);
                if (r == hipSuccess) q.occ_pinned = nullptr;
            } else {
                // pageable: the copy returns once the data has left q.occ
                r = hipMemcpyAsync(occ_dev, q.occ.data(), n_occ, hipMemcpyHostToDevice, e->xfer);
                if (r == hipSuccess) r = hipStreamSynchronize(e->xfer);
            }
        }
        if (r == hipSuccess) r = hipEventRecord(g.ev, e->xfer);
        if (r != hipSuccess) {
            e->mem.release(occ_dev);
            if (g.ev) e->ev_spare.push_back(g.ev);
            return fail(OMAP_ERR_HIP, "occupancy upload: %s", hipGetErrorString(r));
        }
        e->waiting.pop_front();
        query_release_occ(e, q);
        e->reserved += g.reserve;
        e->staged.push_back(g);
    }
    return OMAP_OK;
}

// Copies the per-slot counts that tell which mazes have nothing scheduled for
// the next round (active: no listed tile; dense: no change in the last round).
static omap_status_t engine_snapshot(omap_engine_s* e) {
    Solver& sv = e->solver;
    Snapshot& sn = e->snap[e->snap_next];
    if (!sn.counts) {
        HIP_TRY(hipHostMalloc((void**)&sn.counts, sizeof(int32_t) * sv.cap_slots, hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&sn.ev, hipEventDisableTiming));
    }
    const int64_t r = sv.next_round;
    // (with one slot the kernels keep only the list count, which is that slot's)
    const int32_t* src = sv.opt.dense     ? sv.d_dchg + (size_t)((r + 2) % 3) * sv.cap_slots
                         : sv.cap_slots > 1 ? sv.d_sched + (size_t)(r % 3) * sv.cap_slots
                                            : sv.d_count + r % 3;
    HIP_TRY(hipMemcpyAsync(sn.counts, src, sizeof(int32_t) * sv.cap_slots, hipMemcpyDeviceToHost, sv.stream));
    HIP_TRY(hipEventRecord(sn.ev, sv.stream));
    sn.round = r;
    sn.busy = true;
    e->snap_next ^= 1;
    return OMAP_OK;
}

// A completed snapshot: running mazes that had rounds before it and nothing
// scheduled in it have converged (a converged maze is never visited again,
// so the verdict cannot go stale while other mazes run on).
static void engine_take_snapshot(omap_engine_s* e, Snapshot& sn) {
    std::vector<int64_t> keep;
    for (int64_t id : e->running) {
        const Query& q = e->queries[id];
        const Slot& s = e->solver.slots[q.slot];
        if (s.first_round < sn.round && sn.counts[q.slot] == 0) e->converged.push_back(id);
        else keep.push_back(id);
    }
    e->running.swap(keep);
    sn.busy = false;
}

// Phase 1 of a retirement: finalize every converged maze and compute the
// lengths and offsets of all their paths.
static omap_status_t retire_begin(omap_engine_s* e) {
    Solver& sv = e->solver;
    Retirement& R = e->ret;
    R.ids.swap(e->converged);
    e->converged.clear();
    R.slots.clear();
    std::vector<int32_t> tslot, trc;
    for (int64_t id : R.ids) {
        const Query& q = e->queries[id];
        R.slots.push_back(q.slot);
        const int32_t nt = (int32_t)(q.tgt.size() / 2);
        tslot.insert(tslot.end(), nt, q.slot);
        trc.insert(trc.end(), q.tgt.begin(), q.tgt.end());
    }
    R.n = (int32_t)tslot.size();
    if (!R.h_min) {
        HIP_TRY(hipHostMalloc((void**)&R.h_min, sizeof(int32_t) * sv.cap_slots, hipHostMallocDefault));
        HIP_TRY(hipHostMalloc((void**)&R.h_reached, sizeof(unsigned long long) * sv.cap_slots, hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&R.ev, hipEventDisableTiming));
    }
    OK_TRY(sv.finalize_enqueue(R.slots, R.h_min, R.h_reached));
    // device layout: tslot | trc | len | off
    const size_t n = (size_t)R.n;
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    char* base = nullptr;
    OK_TRY(sv.scratch(up(4 * (n + 1)) + up(8 * (n + 1)) + up(4 * (n + 1)) + up(8 * (n + 1)), &base));
    int32_t* d_tslot = reinterpret_cast<int32_t*>(base);
    int32_t* d_trc = reinterpret_cast<int32_t*>(base + up(4 * (n + 1)));
    int32_t* d_len = reinterpret_cast<int32_t*>(base + up(4 * (n + 1)) + up(8 * (n + 1)));
    int64_t* d_off = reinterpret_cast<int64_t*>(base + 2 * up(4 * (n + 1)) + up(8 * (n + 1)));
    if (n > 0) {
        OK_TRY(sv.upload(d_tslot, tslot.data(), 4 * n));
        OK_TRY(sv.upload(d_trc, trc.data(), 8 * n));
        HIP_TRY(launch_path_lengths(sv.d_mazes, d_tslot, d_trc, R.n, sv.vparity(), d_len, sv.stream));
    }
    HIP_TRY(launch_scan_offsets(d_len, R.n, d_off, sv.stream));
    OK_TRY(R.h_lo.reserve(lo_offsets_at(n) + 8 * (n + 1)));
    if (n > 0) HIP_TRY(hipMemcpyAsync(R.h_lo.p, d_len, 4 * n, hipMemcpyDeviceToHost, sv.stream));
    HIP_TRY(hipMemcpyAsync(R.h_lo.p + lo_offsets_at(n), d_off, 8 * (n + 1), hipMemcpyDeviceToHost, sv.stream));
    HIP_TRY(hipEventRecord(R.ev, sv.stream));
    R.phase = 1;
    return OMAP_OK;
}

// Phase 2: with the path sizes known, walk every path and copy paths,
// visit counters and kept activity maps to pinned host memory, all on the
// transfer stream (after phase 1), so that the rounds of the mazes still
// running go on meanwhile: the retiring mazes' buffers are no longer written.
static omap_status_t retire_paths(omap_engine_s* e) {
    Solver& sv = e->solver;
    Retirement& R = e->ret;
    sv.finalize_apply(R.slots, R.h_min, R.h_reached);
    const size_t n = (size_t)R.n;
    const int64_t* h_off = reinterpret_cast<const int64_t*>(R.h_lo.p + lo_offsets_at(n));
    R.total = h_off[n];
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    char* base = nullptr;
    OK_TRY(sv.scratch(up(4 * (n + 1)) + up(8 * (n + 1)) + up(4 * (n + 1)) + up(8 * (n + 1)), &base));
    const int32_t* d_tslot = reinterpret_cast<const int32_t*>(base);
    const int32_t* d_trc = reinterpret_cast<const int32_t*>(base + up(4 * (n + 1)));
    const int32_t* d_len = reinterpret_cast<const int32_t*>(base + up(4 * (n + 1)) + up(8 * (n + 1)));
    const int64_t* d_off = reinterpret_cast<const int64_t*>(base + 2 * up(4 * (n + 1)) + up(8 * (n + 1)));
    hipStream_t xs = e->xfer;
    HIP_TRY(hipStreamWaitEvent(xs, R.ev, 0));
    if ((size_t)R.total > R.cells_cap) {
        const size_t want = std::max<size_t>((size_t)R.total, R.cells_cap * 2);
        HIP_TRY(hipStreamSynchronize(xs));
        if (R.d_cells) (void)hipFree(R.d_cells);
        R.d_cells = nullptr;
        R.cells_cap = 0;
        HIP_TRY(hipMalloc(&R.d_cells, 4 * want));
        R.cells_cap = want;
    }
    if (n > 0 && R.total > 0)
        HIP_TRY(launch_walk(sv.d_mazes, d_tslot, d_trc, R.n, sv.vparity(), d_len, d_off, R.d_cells, xs));
    // host layout: last_round | visits | cell visits | cells | activity maps
    const size_t b_lr = up(4 * (size_t)sv.cap_slots), b_v = up(8 * (size_t)sv.cap_slots * kSpread);
    size_t act_bytes = 0;
    R.act_off.assign(R.ids.size(), -1);
    const size_t cells_at = b_lr + 2 * b_v, act_at = cells_at + up(4 * (size_t)R.total);
    for (size_t i = 0; i < R.ids.size(); ++i) {
        const Query& q = e->queries[R.ids[i]];
        if (!(q.flags & OMAP_QUERY_KEEP_ACTIVITY)) continue;
        R.act_off[i] = (int64_t)(act_at + act_bytes);
        act_bytes += up(4 * (size_t)q.H * q.W);
    }
    OK_TRY(R.h_out.reserve(act_at + act_bytes));
    // (the counters of the retiring slots no longer change; the other
    // slots' entries of this snapshot are not used)
    HIP_TRY(hipMemcpyAsync(R.h_out.p, sv.d_last_round, 4 * (size_t)sv.cap_slots, hipMemcpyDeviceToHost, xs));
    HIP_TRY(hipMemcpyAsync(R.h_out.p + b_lr, sv.d_visits, 8 * (size_t)sv.cap_slots * kSpread, hipMemcpyDeviceToHost,
                           xs));
    HIP_TRY(hipMemcpyAsync(R.h_out.p + b_lr + b_v, sv.d_cell_visits, 8 * (size_t)sv.cap_slots * kSpread,
                           hipMemcpyDeviceToHost, xs));
    // each query's cells straight into a block of the result pool that
    // omap_engine_fetch copies out and frees (else into h_out)
    R.cells_block.assign(R.ids.size(), nullptr);
    int64_t t0 = 0;
    for (size_t i = 0; i < R.ids.size(); ++i) {
        const int64_t nt = (int64_t)(e->queries[R.ids[i]].tgt.size() / 2);
        const int64_t a = h_off[t0], b = h_off[t0 + nt];
        t0 += nt;
        if (b <= a) continue;
        void* blk = e->res_pool.alloc(4 * (size_t)(b - a));
        R.cells_block[i] = blk;
        HIP_TRY(hipMemcpyAsync(blk ? blk : R.h_out.p + cells_at + 4 * a, R.d_cells + a, 4 * (size_t)(b - a),
                               hipMemcpyDeviceToHost, xs));
    }
    if (act_bytes > 0) {
        if (act_bytes > R.act_cap) {
            HIP_TRY(hipStreamSynchronize(xs));
            if (R.d_act) (void)hipFree(R.d_act);
            R.d_act = nullptr;
            R.act_cap = 0;
            HIP_TRY(hipMalloc(&R.d_act, act_bytes));
            R.act_cap = act_bytes;
        }
        for (size_t i = 0; i < R.ids.size(); ++i) {
            if (R.act_off[i] < 0) continue;
            const Query& q = e->queries[R.ids[i]];
            const Slot& s = sv.slots[q.slot];
            int32_t* d = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(R.d_act) + (R.act_off[i] - act_at));
            HIP_TRY(launch_activity(sv.d_mazes, q.slot, q.H, q.W, sv.vparity(), (int32_t)((int64_t)s.K - s.layers - 1),
                                    d, q.W, xs));
            HIP_TRY(hipMemcpyAsync(R.h_out.p + R.act_off[i], d, 4 * (size_t)q.H * q.W, hipMemcpyDeviceToHost, xs));
        }
    }
    HIP_TRY(hipEventRecord(R.ev, xs));
    R.phase = 2;
    return OMAP_OK;
}

// Phase 3: results to the queries, slots and memory freed.
static omap_status_t retire_finish(omap_engine_s* e) {
    Solver& sv = e->solver;
    Retirement& R = e->ret;
    const size_t n = (size_t)R.n;
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t b_lr = up(4 * (size_t)sv.cap_slots), b_v = up(8 * (size_t)sv.cap_slots * kSpread);
    const int32_t* h_len = reinterpret_cast<const int32_t*>(R.h_lo.p);
    const int64_t* h_off = reinterpret_cast<const int64_t*>(R.h_lo.p + lo_offsets_at(n));
    const int32_t* h_cells = reinterpret_cast<const int32_t*>(R.h_out.p + b_lr + 2 * b_v);
    const int32_t* h_lr = reinterpret_cast<const int32_t*>(R.h_out.p);
    const int64_t* h_v = reinterpret_cast<const int64_t*>(R.h_out.p + b_lr);
    const int64_t* h_cv = reinterpret_cast<const int64_t*>(R.h_out.p + b_lr + b_v);
    sv.h_last_round.assign(h_lr, h_lr + sv.cap_slots);
    sv.h_visits.assign(h_v, h_v + (size_t)sv.cap_slots * kSpread);
    sv.h_cell_visits.assign(h_cv, h_cv + (size_t)sv.cap_slots * kSpread);
    int64_t t0 = 0;
    for (size_t i = 0; i < R.ids.size(); ++i) {
        Query& q = e->queries[R.ids[i]];
        const int32_t k = R.slots[i];
        const int64_t nt = (int64_t)(q.tgt.size() / 2);
        q.len.assign(h_len + t0, h_len + t0 + nt);
        q.off.resize((size_t)nt + 1);
        for (int64_t j = 0; j <= nt; ++j) q.off[j] = h_off[t0 + j] - h_off[t0];
        q.n_cells = h_off[t0 + nt] - h_off[t0];
        if (R.cells_block[i]) q.cells_pinned = static_cast<int32_t*>(R.cells_block[i]);
        else q.cells.assign(h_cells + h_off[t0], h_cells + h_off[t0 + nt]);
        if (R.act_off[i] >= 0) {
            const int32_t* a = reinterpret_cast<const int32_t*>(R.h_out.p + R.act_off[i]);
            q.activity.assign(a, a + (size_t)q.H * q.W);
        }
        t0 += nt;
        OK_TRY(sv.info(k, &q.info, /*counters_read=*/true));
        OK_TRY(sv.remove(k));
        q.slot = -1;
        q.state = OMAP_QUERY_DONE;
        ++e->done_total;
        e->completed.push_back(q.id);
    }
    R.ids.clear();
    R.slots.clear();
    R.phase = 0;
    return OMAP_OK;
}

static bool event_done(hipEvent_t ev, bool wait) {
    if (wait) return hipEventSynchronize(ev) == hipSuccess;
    const hipError_t e = hipEventQuery(ev);
    if (e == hipSuccess) return true;
    (void)hipGetLastError();
    return false;
}

// Advances everything that completed on the device: snapshots, then the
// retirement phases.  With wait, blocks until the current retirement phase
// (if any) has completed.
static omap_status_t engine_progress(omap_engine_s* e, bool wait) {
    for (int k = 0; k < 2; ++k) {
        Snapshot& sn = e->snap[e->snap_next ^ k];   // the older one first
        if (sn.busy && event_done(sn.ev, false)) engine_take_snapshot(e, sn);
    }
    for (;;) {
        Retirement& R = e->ret;
        if (R.phase == 0) {
            if (e->converged.empty()) return OMAP_OK;
            OK_TRY(retire_begin(e));
        }
        if (!event_done(R.ev, wait)) return OMAP_OK;
        if (R.phase == 1) OK_TRY(retire_paths(e));
        else OK_TRY(retire_finish(e));
    }
}
}  // namespace omap

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

using namespace omap;

#define API_GUARD_BEGIN try {
#define API_GUARD_END                                                              \
    }                                                                              \
    catch (const std::bad_alloc&) {                                                \
        return fail(OMAP_ERR_OUT_OF_MEMORY, "host allocation failed");             \
    }                                                                              \
    catch (...) {                                                                  \
        return fail(OMAP_ERR_HIP, "unexpected exception");                         \
    }

extern "C" {

const char* omap_version(void) { return "omap-gfx950 0.1"; }

omap_status_t omap_resolve_options(const omap_options* options, omap_options* resolved) {
    if (!resolved) return fail(OMAP_ERR_INVALID_ARG, "resolved is NULL");
    Options r;
    OK_TRY(resolve_options(options, &r));
    resolved->temporal_depth = r.T;
    resolved->tile_rows = r.TH;
    resolved->schedule = r.bits ? OMAP_SCHEDULE_BITS : (r.dense ? OMAP_SCHEDULE_DENSE : OMAP_SCHEDULE_ACTIVE);
    resolved->check_interval = r.check;
    resolved->lane_columns = r.bits ? 0 : r.C;
    resolved->round_launch = r.graph ? OMAP_LAUNCH_GRAPH : OMAP_LAUNCH_PER_ROUND;
    return OMAP_OK;
}

const char* omap_last_error(void) { return g_last_error.c_str(); }

const char* omap_status_string(omap_status_t s) {
    switch (s) {
        case OMAP_OK: return "OMAP_OK";
        case OMAP_ERR_INVALID_ARG: return "OMAP_ERR_INVALID_ARG";
        case OMAP_ERR_TOO_LARGE: return "OMAP_ERR_TOO_LARGE";
        case OMAP_ERR_SOURCE_OUT_OF_BOUNDS: return "OMAP_ERR_SOURCE_OUT_OF_BOUNDS";
        case OMAP_ERR_SOURCE_ON_OBSTACLE: return "OMAP_ERR_SOURCE_ON_OBSTACLE";
        case OMAP_ERR_NO_SOURCES: return "OMAP_ERR_NO_SOURCES";
        case OMAP_ERR_TARGET_OUT_OF_BOUNDS: return "OMAP_ERR_TARGET_OUT_OF_BOUNDS";
        case OMAP_ERR_NOT_PROPAGATED: return "OMAP_ERR_NOT_PROPAGATED";
        case OMAP_ERR_BUFFER_TOO_SMALL: return "OMAP_ERR_BUFFER_TOO_SMALL";
        case OMAP_ERR_OUT_OF_MEMORY: return "OMAP_ERR_OUT_OF_MEMORY";
        case OMAP_ERR_HIP: return "OMAP_ERR_HIP";
        case OMAP_ERR_NOT_FOUND: return "OMAP_ERR_NOT_FOUND";
        case OMAP_ERR_BUSY: return "OMAP_ERR_BUSY";
    }
    return "OMAP_ERR_UNKNOWN";
}

omap_status_t omap_plan_create(omap_plan_t* out, int32_t height, int32_t width,
                               const uint8_t* occupancy_dev, const int32_t* sources_host,
                               int32_t n_sources, const int32_t* targets_host, int32_t n_targets,
                               const omap_options* opts, void* stream) {
    API_GUARD_BEGIN
    if (!out) return fail(OMAP_ERR_INVALID_ARG, "out is NULL");
    OK_TRY(validate_problem(height, width, occupancy_dev, sources_host, n_sources, targets_host, n_targets));
    Options o;
    OK_TRY(resolve_options(opts, &o));
    std::unique_ptr<omap_plan_s> p(new omap_plan_s());
    HIP_TRY(hipGetDevice(&p->device));
    const Geometry g = make_geometry(height, width, o);
    OK_TRY(p->solver.init(static_cast<hipStream_t>(stream), o, &p->mem, 1, g.tiles_x * g.tiles_y));
    OK_TRY(p->solver.add(height, width, occupancy_dev, sources_host, n_sources, targets_host, n_targets, &p->slot));
    *out = p.release();
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_plan_load(omap_plan_t plan, const uint8_t* occupancy_dev,
                             const int32_t* sources_host, int32_t n_sources,
                             const int32_t* targets_host, int32_t n_targets) {
    API_GUARD_BEGIN
    if (!plan) return fail(OMAP_ERR_INVALID_ARG, "plan is NULL");
    plan->propagated = false;
    return plan->solver.pack(plan->slot, occupancy_dev, sources_host, n_sources, targets_host, n_targets);
    API_GUARD_END
}

static void fill_info_basic(omap_propagate_info* info) { std::memset(info, 0, sizeof *info); }

omap_status_t omap_propagate(omap_plan_t plan, int64_t max_layers, omap_propagate_info* info) {
    API_GUARD_BEGIN
    if (!plan) return fail(OMAP_ERR_INVALID_ARG, "plan is NULL");
    Solver& s = plan->solver;
    plan->propagated = false;
    OK_TRY(s.reset_schedule());
    OK_TRY(s.start(plan->slot, max_layers));
    OK_TRY(s.run_to_convergence());
    plan->propagated = true;
    if (info) {
        fill_info_basic(info);
        OK_TRY(s.info(plan->slot, info));
    }
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_get_activity(omap_plan_t plan, int32_t* dst_dev, int64_t dst_pitch_elems) {
    API_GUARD_BEGIN
    if (!plan) return fail(OMAP_ERR_INVALID_ARG, "plan is NULL");
    if (!plan->propagated) return fail(OMAP_ERR_NOT_PROPAGATED, "call omap_propagate first");
    return plan->solver.activity(plan->slot, dst_dev, dst_pitch_elems);
    API_GUARD_END
}

omap_status_t omap_extract_paths(omap_plan_t plan, int32_t* len_dev, int64_t* offsets_dev,
                                 int32_t* cells_dev, int64_t cells_capacity,
                                 int64_t* cells_needed_host) {
    API_GUARD_BEGIN
    if (!plan) return fail(OMAP_ERR_INVALID_ARG, "plan is NULL");
    if (!plan->propagated) return fail(OMAP_ERR_NOT_PROPAGATED, "call omap_propagate first");
    const int32_t nt = (int32_t)(plan->solver.slots[plan->slot].tgt.size() / 2);
    if (!offsets_dev || (nt > 0 && !len_dev)) return fail(OMAP_ERR_INVALID_ARG, "len/offsets pointer is NULL");
    std::vector<int32_t> one{plan->slot};
    return plan->solver.extract(one, len_dev, offsets_dev, cells_dev, cells_capacity, cells_needed_host, false);
    API_GUARD_END
}

static omap_status_t walk_mode(const omap_walk_options* w, int* mode, uint64_t* seed) {
    *mode = 0;
    *seed = 0;
    if (!w) return OMAP_OK;
    if (w->mode != OMAP_WALK_FIRST_MAX && w->mode != OMAP_WALK_RANDOM_TIES && w->mode != OMAP_WALK_EUCLIDEAN)
        return fail(OMAP_ERR_INVALID_ARG, "walk mode %d", w->mode);
    *mode = w->mode;
    *seed = w->seed;
    return OMAP_OK;
}

omap_status_t omap_extract_paths_ex(omap_plan_t plan, const omap_walk_options* walk, int32_t* len_dev,
                                    int64_t* offsets_dev, int32_t* cells_dev, int64_t cells_capacity,
                                    int64_t* cells_needed_host, int32_t* source_index_dev) {
    API_GUARD_BEGIN
    if (!plan) return fail(OMAP_ERR_INVALID_ARG, "plan is NULL");
    int mode = 0;
    uint64_t seed = 0;
    OK_TRY(walk_mode(walk, &mode, &seed));
    if (!plan->propagated) return fail(OMAP_ERR_NOT_PROPAGATED, "call omap_propagate first");
    const int32_t nt = (int32_t)(plan->solver.slots[plan->slot].tgt.size() / 2);
    if (!offsets_dev || (nt > 0 && !len_dev)) return fail(OMAP_ERR_INVALID_ARG, "len/offsets pointer is NULL");
    std::vector<int32_t> one{plan->slot};
    return plan->solver.extract(one, len_dev, offsets_dev, cells_dev, cells_capacity, cells_needed_host, false,
                                mode, seed, source_index_dev);
    API_GUARD_END
}

// ---- allocation-free path extraction ----------------------------------------

// Per-target staging of omap_extract_paths_noalloc: slot ids, then (row, col)
// pairs.  Each device holds its own copy for the life of the process; host
// code uses only the device address obtained for it below.
static __device__ __align__(256) int32_t scratch[3 * OMAP_NOALLOC_MAX_TARGETS];

static std::mutex g_scratch_mu;
static int32_t* g_scratch_ptr[1024];   // per device id, once looked up

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
static omap_status_t noalloc_scratch(int32_t** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 1024) return fail(OMAP_ERR_HIP, "device id %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(OMAP_ERR_HIP, "no device address for the extraction staging");
        g_scratch_ptr[dev] = static_cast<int32_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return OMAP_OK;
}

static omap_status_t extract_noalloc(omap_plan_t plan, int32_t* len_dev, int64_t* offsets_dev, int32_t* cells_dev,
                                     int64_t cells_capacity, int64_t* cells_needed_host) {
    Solver& sv = plan->solver;
    const Slot& s = sv.slots[plan->slot];
    const int32_t n = (int32_t)(s.tgt.size() / 2);
    if (n > OMAP_NOALLOC_MAX_TARGETS)
        return fail(OMAP_ERR_TOO_LARGE, "%d targets, the allocation-free extraction takes at most %d", n,
                    OMAP_NOALLOC_MAX_TARGETS);
    int32_t* d_scratch = nullptr;
    OK_TRY(noalloc_scratch(&d_scratch));
    int32_t* d_tslot = d_scratch;
    int32_t* d_trc = d_scratch + OMAP_NOALLOC_MAX_TARGETS;
    void* staged = nullptr;   // targets copied through the plan's pinned pool when they fit
    if (n > 0) {
        HIP_TRY(launch_fill(d_tslot, n, plan->slot, sv.stream));
        const size_t b = sizeof(int32_t) * 2 * (size_t)n;
        staged = sv.pin.alloc(b);
        if (staged) std::memcpy(staged, s.tgt.data(), b);
        const hipError_t e = hipMemcpyAsync(d_trc, staged ? staged : s.tgt.data(), b, hipMemcpyHostToDevice, sv.stream);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(sv.stream);
            if (staged) sv.pin.release_now(staged);
            HIP_TRY(e);
        }
        HIP_TRY(launch_path_lengths(sv.d_mazes, d_tslot, d_trc, n, sv.vparity(), len_dev, sv.stream));
    }
    HIP_TRY(launch_scan_offsets(len_dev, n, offsets_dev, sv.stream));
    HIP_TRY(hipMemcpyAsync(sv.h_pinned, offsets_dev + n, sizeof(int64_t), hipMemcpyDeviceToHost, sv.stream));
    const hipError_t sync = hipStreamSynchronize(sv.stream);   // the staging copy above has completed too
    if (staged) sv.pin.release_now(staged);
    HIP_TRY(sync);
    int64_t total = 0;
    std::memcpy(&total, sv.h_pinned, sizeof total);
    if (cells_needed_host) *cells_needed_host = total;
    if (cells_capacity < total || (total > 0 && cells_dev == nullptr))
        return fail(OMAP_ERR_BUFFER_TOO_SMALL, "paths need %lld cells, capacity %lld", (long long)total,
                    (long long)cells_capacity);
    if (n > 0 && total > 0)
        HIP_TRY(launch_walk(sv.d_mazes, d_tslot, d_trc, n, sv.vparity(), len_dev, offsets_dev, cells_dev, sv.stream));
    HIP_TRY(hipStreamSynchronize(sv.stream));
    return OMAP_OK;
}

omap_status_t omap_extract_paths_noalloc(omap_plan_t plan, int32_t* len_dev, int64_t* offsets_dev,
                                         int32_t* cells_dev, int64_t cells_capacity,
                                         int64_t* cells_needed_host) {
    API_GUARD_BEGIN
    if (!plan) return fail(OMAP_ERR_INVALID_ARG, "plan is NULL");
    if (!plan->propagated) return fail(OMAP_ERR_NOT_PROPAGATED, "call omap_propagate first");
    const int32_t nt = (int32_t)(plan->solver.slots[plan->slot].tgt.size() / 2);
    if (!offsets_dev || (nt > 0 && !len_dev)) return fail(OMAP_ERR_INVALID_ARG, "len/offsets pointer is NULL");
    // the staging array is looked up (and used) on the plan's device
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != plan->device) HIP_TRY(hipSetDevice(plan->device));
    const omap_status_t st = extract_noalloc(plan, len_dev, offsets_dev, cells_dev, cells_capacity, cells_needed_host);
    if (cur != plan->device) {
        const hipError_t e = hipSetDevice(cur);
        if (st == OMAP_OK && e != hipSuccess) return fail(OMAP_ERR_HIP, "hipSetDevice: %s", hipGetErrorString(e));
    }
    return st;
    API_GUARD_END
}

omap_status_t omap_plan_destroy(omap_plan_t plan) {
    API_GUARD_BEGIN
    if (!plan) return OMAP_OK;
    (void)hipStreamSynchronize(plan->solver.stream);
    delete plan;
    return OMAP_OK;
    API_GUARD_END
}

// ---- batch -----------------------------------------------------------------

omap_status_t omap_batch_create(omap_batch_t* out, const omap_maze_desc* mazes, int32_t n_mazes,
                                const omap_options* opts, void* stream) {
    API_GUARD_BEGIN
    if (!out || !mazes || n_mazes < 1) return fail(OMAP_ERR_INVALID_ARG, "need out and n_mazes >= 1");
    Options o;
    OK_TRY(resolve_options(opts, &o, Use::kMany));
    int64_t tiles = 0;
    for (int32_t i = 0; i < n_mazes; ++i) {
        const omap_maze_desc& d = mazes[i];
        omap_status_t st = validate_problem(d.height, d.width, d.occupancy_dev, d.sources_host,
                                            d.n_sources, d.targets_host, d.n_targets);
        if (st != OMAP_OK) {
            g_last_error += " (maze " + std::to_string(i) + ")";
            return st;
        }
        const Geometry g = make_geometry(d.height, d.width, o);
        tiles += (int64_t)g.tiles_x * g.tiles_y;
    }
    if (tiles >= (int64_t(1) << 31)) return fail(OMAP_ERR_TOO_LARGE, "too many tiles");
    int64_t bytes = 0;
    for (int32_t i = 0; i < n_mazes; ++i)
        bytes += maze_device_bytes(mazes[i].height, mazes[i].width, o) + 8 * (int64_t)mazes[i].n_sources + 1024;
    std::unique_ptr<omap_batch_s> b(new omap_batch_s());
    if (!b->mem.init((size_t)bytes))
        return fail(OMAP_ERR_OUT_OF_MEMORY, "batch buffers (%lld bytes)", (long long)bytes);
    OK_TRY(b->solver.init(static_cast<hipStream_t>(stream), o, &b->mem, n_mazes, (int32_t)tiles));
    // one clear of the whole arena (before the masks are packed into it):
    // every maze starts with zero activity
    HIP_TRY(hipMemsetAsync(b->mem.base(), 0, b->mem.size(), b->solver.stream));
    OK_TRY(b->solver.add_many(mazes, n_mazes, &b->slots));
    for (int32_t k : b->slots) b->solver.slots[k].cleared = true;
    int32_t bad = -1;
    omap_status_t st = b->solver.commit(b->slots, &bad);
    if (st != OMAP_OK) {
        g_last_error += " (maze " + std::to_string(bad) + ")";
        return st;
    }
    *out = b.release();
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_batch_propagate(omap_batch_t batch, const int64_t* max_layers_host,
                                   omap_propagate_info* infos_host) {
    API_GUARD_BEGIN
    if (!batch) return fail(OMAP_ERR_INVALID_ARG, "batch is NULL");
    Solver& s = batch->solver;
    batch->propagated = false;
    OK_TRY(s.reset_schedule());
    std::vector<int64_t> Ls(batch->slots.size(), (int64_t)OMAP_AUTO_LAYERS);
    if (max_layers_host) Ls.assign(max_layers_host, max_layers_host + batch->slots.size());
    OK_TRY(s.start_many(batch->slots, Ls.data()));
    OK_TRY(s.run_to_convergence());
    batch->propagated = true;
    if (infos_host) {
        OK_TRY(s.finalize(batch->slots));
        for (size_t i = 0; i < batch->slots.size(); ++i) {
            fill_info_basic(&infos_host[i]);
            OK_TRY(s.info(batch->slots[i], &infos_host[i]));
        }
    }
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_batch_get_activity(omap_batch_t batch, int32_t index, int32_t* dst_dev,
                                      int64_t dst_pitch_elems) {
    API_GUARD_BEGIN
    if (!batch) return fail(OMAP_ERR_INVALID_ARG, "batch is NULL");
    if (index < 0 || index >= (int32_t)batch->slots.size())
        return fail(OMAP_ERR_INVALID_ARG, "maze index %d out of range", index);
    if (!batch->propagated) return fail(OMAP_ERR_NOT_PROPAGATED, "call omap_batch_propagate first");
    return batch->solver.activity(batch->slots[index], dst_dev, dst_pitch_elems);
    API_GUARD_END
}

omap_status_t omap_batch_extract_paths(omap_batch_t batch, int32_t* len_dev, int64_t* offsets_dev,
                                       int32_t* cells_dev, int64_t cells_capacity,
                                       int64_t* cells_needed_host) {
    API_GUARD_BEGIN
    if (!batch) return fail(OMAP_ERR_INVALID_ARG, "batch is NULL");
    if (!batch->propagated) return fail(OMAP_ERR_NOT_PROPAGATED, "call omap_batch_propagate first");
    if (!offsets_dev || !len_dev) return fail(OMAP_ERR_INVALID_ARG, "len/offsets pointer is NULL");
    return batch->solver.extract(batch->slots, len_dev, offsets_dev, cells_dev, cells_capacity,
                                 cells_needed_host, false);
    API_GUARD_END
}

omap_status_t omap_batch_extract_paths_ex(omap_batch_t batch, const omap_walk_options* walk,
                                          int32_t* len_dev, int64_t* offsets_dev, int32_t* cells_dev,
                                          int64_t cells_capacity, int64_t* cells_needed_host,
                                          int32_t* source_index_dev) {
    API_GUARD_BEGIN
    if (!batch) return fail(OMAP_ERR_INVALID_ARG, "batch is NULL");
    int mode = 0;
    uint64_t seed = 0;
    OK_TRY(walk_mode(walk, &mode, &seed));
    if (!batch->propagated) return fail(OMAP_ERR_NOT_PROPAGATED, "call omap_batch_propagate first");
    if (!offsets_dev || !len_dev) return fail(OMAP_ERR_INVALID_ARG, "len/offsets pointer is NULL");
    return batch->solver.extract(batch->slots, len_dev, offsets_dev, cells_dev, cells_capacity,
                                 cells_needed_host, false, mode, seed, source_index_dev);
    API_GUARD_END
}

omap_status_t omap_batch_destroy(omap_batch_t batch) {
    API_GUARD_BEGIN
    if (!batch) return OMAP_OK;
    (void)hipStreamSynchronize(batch->solver.stream);
    delete batch;
    return OMAP_OK;
    API_GUARD_END
}

// ---- serving engine ----------------------------------------------------------

omap_status_t omap_engine_create(omap_engine_t* out, int64_t memory_budget_bytes, int32_t max_slots,
                                 const omap_options* opts, void* stream) {
    API_GUARD_BEGIN
    if (!out || memory_budget_bytes < (1 << 20) || max_slots < 1)
        return fail(OMAP_ERR_INVALID_ARG, "need out, budget >= 1 MiB and max_slots >= 1");
    Options o;
    OK_TRY(resolve_options(opts, &o, Use::kMany));
    std::unique_ptr<omap_engine_s> e(new omap_engine_s());
    if (!e->mem.init((size_t)memory_budget_bytes))
        return fail(OMAP_ERR_OUT_OF_MEMORY, "engine budget of %lld bytes", (long long)memory_budget_bytes);
    // pinned copies of queued occupancy grids: a quarter of the budget, 16 MiB .. 4 GiB
    const int64_t pool = std::min<int64_t>(std::max<int64_t>(memory_budget_bytes / 4, 16 << 20), int64_t(4) << 30);
    if (!e->occ_pool.init((size_t)pool)) return fail(OMAP_ERR_OUT_OF_MEMORY, "pinned staging of %lld bytes", (long long)pool);
    if (!e->res_pool.init((size_t)pool)) return fail(OMAP_ERR_OUT_OF_MEMORY, "pinned results of %lld bytes", (long long)pool);
    e->budget = memory_budget_bytes;
    e->max_slots = max_slots;
    // tile ids: enough for the whole budget filled with the smallest mazes
    const int64_t per_tile = (int64_t)o.TH * o.TW * 8;
    int64_t cap_tiles = memory_budget_bytes / per_tile + 4 * (int64_t)max_slots + 64;
    if (cap_tiles > (int64_t(1) << 28)) cap_tiles = int64_t(1) << 28;
    OK_TRY(e->solver.init(static_cast<hipStream_t>(stream), o, &e->mem, max_slots, (int32_t)cap_tiles,
                          size_t(16) << 20));
    HIP_TRY(hipStreamCreateWithFlags(&e->xfer, hipStreamNonBlocking));
    *out = e.release();
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_engine_submit_ex(omap_engine_t engine, int32_t height, int32_t width,
                                    const uint8_t* occupancy_host, const int32_t* sources_host,
                                    int32_t n_sources, const int32_t* targets_host, int32_t n_targets,
                                    int64_t max_layers, uint32_t flags, int64_t* query_id) {
    API_GUARD_BEGIN
    if (!engine || !query_id) return fail(OMAP_ERR_INVALID_ARG, "engine/query_id is NULL");
    if (flags & ~uint32_t(OMAP_QUERY_KEEP_ACTIVITY)) return fail(OMAP_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    OK_TRY(validate_problem(height, width, occupancy_host, sources_host, n_sources, targets_host, n_targets));
    if (max_layers < -1) return fail(OMAP_ERR_INVALID_ARG, "max_layers must be >= 0 or OMAP_AUTO_LAYERS");
    if (max_layers >= 0 && max_layers + 1 > 0x7fffffffLL) return fail(OMAP_ERR_TOO_LARGE, "L + 1 >= 2^31");
    Query q;
    q.id = engine->next_id;
    q.H = height;
    q.W = width;
    q.src.assign(sources_host, sources_host + 2 * n_sources);
    if (n_targets > 0) q.tgt.assign(targets_host, targets_host + 2 * n_targets);
    q.L = max_layers;
    q.flags = flags;
    q.bytes = query_bytes(q, engine->solver.opt);
    if (q.bytes > (int64_t)engine->mem.size())
        return fail(OMAP_ERR_OUT_OF_MEMORY, "query needs %lld bytes, budget is %lld", (long long)q.bytes,
                    (long long)engine->mem.size());
    const Geometry g = make_geometry(height, width, engine->solver.opt);
    if ((int64_t)g.tiles_x * g.tiles_y > engine->solver.cap_tiles)
        return fail(OMAP_ERR_OUT_OF_MEMORY, "query has more tiles than the engine's tile table");
    const size_t n_occ = (size_t)height * width;
    engine->occ_pool.reap(false);
    void* pinned = engine->occ_pool.alloc(n_occ);
    if (pinned) {
        host_copy(pinned, occupancy_host, n_occ);
        q.occ_pinned = static_cast<uint8_t*>(pinned);
    } else {
        q.occ.assign(occupancy_host, occupancy_host + n_occ);
    }
    ++engine->next_id;
    *query_id = q.id;
    engine->waiting.push_back(q.id);
    engine->queries.emplace(q.id, std::move(q));
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_engine_submit(omap_engine_t engine, int32_t height, int32_t width,
                                 const uint8_t* occupancy_host, const int32_t* sources_host,
                                 int32_t n_sources, const int32_t* targets_host, int32_t n_targets,
                                 int64_t max_layers, int64_t* query_id) {
    return omap_engine_submit_ex(engine, height, width, occupancy_host, sources_host, n_sources, targets_host,
                                 n_targets, max_layers, 0, query_id);
}

omap_status_t omap_engine_step(omap_engine_t engine, int32_t rounds, int32_t* n_resident,
                               int64_t* n_done_total) {
    API_GUARD_BEGIN
    if (!engine || rounds < 0) return fail(OMAP_ERR_INVALID_ARG, "engine is NULL or rounds < 0");
    omap_engine_s* e = engine;
    OK_TRY(engine_progress(e, false));
    OK_TRY(engine_admit(e));
    if (!e->running.empty() && rounds > 0) {
        // at most two steps of rounds ahead of the device: wait for the older
        // snapshot before enqueueing more
        Snapshot& old = e->snap[e->snap_next];
        if (old.busy) {
            HIP_TRY(hipEventSynchronize(old.ev));
            engine_take_snapshot(e, old);
        }
        OK_TRY(e->solver.run_rounds(rounds));
        OK_TRY(engine_snapshot(e));
        OK_TRY(engine_progress(e, false));
    } else {
        // nothing to advance: wait for what is in flight so that a caller's
        // loop of steps makes progress
        for (int k = 0; k < 2; ++k) {
            Snapshot& sn = e->snap[e->snap_next ^ k];
            if (sn.busy) {
                HIP_TRY(hipEventSynchronize(sn.ev));
                engine_take_snapshot(e, sn);
            }
        }
        OK_TRY(engine_progress(e, true));
        if (!e->staged.empty()) HIP_TRY(hipEventSynchronize(e->staged.front().ev));
        OK_TRY(engine_admit(e));
    }
    if (n_resident) *n_resident = e->resident();
    if (n_done_total) *n_done_total = e->done_total;
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_engine_completed(omap_engine_t engine, int64_t* ids_host, int32_t capacity, int32_t* n_ids) {
    API_GUARD_BEGIN
    if (!engine || !n_ids || capacity < 0 || (capacity > 0 && !ids_host))
        return fail(OMAP_ERR_INVALID_ARG, "engine, n_ids and ids_host (capacity > 0) are required");
    int32_t n = 0;
    while (n < capacity && !engine->completed.empty()) {
        ids_host[n++] = engine->completed.front();
        engine->completed.pop_front();
    }
    *n_ids = n;
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_engine_poll(omap_engine_t engine, int64_t query_id, int32_t* state) {
    API_GUARD_BEGIN
    if (!engine || !state) return fail(OMAP_ERR_INVALID_ARG, "engine/state is NULL");
    auto it = engine->queries.find(query_id);
    if (it == engine->queries.end()) return fail(OMAP_ERR_NOT_FOUND, "query %lld", (long long)query_id);
    *state = it->second.state;
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_engine_fetch_activity(omap_engine_t engine, int64_t query_id, int32_t* dst_host,
                                         int64_t dst_pitch_elems) {
    API_GUARD_BEGIN
    if (!engine || !dst_host) return fail(OMAP_ERR_INVALID_ARG, "engine/destination is NULL");
    auto it = engine->queries.find(query_id);
    if (it == engine->queries.end()) return fail(OMAP_ERR_NOT_FOUND, "query %lld", (long long)query_id);
    const Query& q = it->second;
    if (q.state != OMAP_QUERY_DONE) return fail(OMAP_ERR_BUSY, "query %lld not finished", (long long)query_id);
    if (!(q.flags & OMAP_QUERY_KEEP_ACTIVITY))
        return fail(OMAP_ERR_INVALID_ARG, "query %lld was not submitted with OMAP_QUERY_KEEP_ACTIVITY",
                    (long long)query_id);
    if (dst_pitch_elems < q.W) return fail(OMAP_ERR_INVALID_ARG, "pitch %lld < width %d", (long long)dst_pitch_elems, q.W);
    for (int32_t r = 0; r < q.H; ++r)
        std::memcpy(dst_host + (int64_t)r * dst_pitch_elems, q.activity.data() + (int64_t)r * q.W,
                    sizeof(int32_t) * q.W);
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_engine_fetch(omap_engine_t engine, int64_t query_id, int32_t* len_host,
                                int64_t* offsets_host, int32_t* cells_host, int64_t cells_capacity,
                                int64_t* cells_needed_host, omap_propagate_info* info_host) {
    API_GUARD_BEGIN
    if (!engine) return fail(OMAP_ERR_INVALID_ARG, "engine is NULL");
    auto it = engine->queries.find(query_id);
    if (it == engine->queries.end()) return fail(OMAP_ERR_NOT_FOUND, "query %lld", (long long)query_id);
    Query& q = it->second;
    if (q.state == OMAP_QUERY_FAILED) {
        const std::string msg = q.error;
        engine->queries.erase(it);
        g_last_error = msg;
        return OMAP_ERR_SOURCE_ON_OBSTACLE;
    }
    if (q.state != OMAP_QUERY_DONE) return fail(OMAP_ERR_BUSY, "query %lld not finished", (long long)query_id);
    const int64_t total = q.off.empty() ? 0 : q.off.back();
    if (cells_needed_host) *cells_needed_host = total;
    if (cells_capacity < total || (total > 0 && !cells_host))
        return fail(OMAP_ERR_BUFFER_TOO_SMALL, "paths need %lld cells", (long long)total);
    const size_t nt = q.tgt.size() / 2;
    if ((nt > 0 && !len_host) || !offsets_host) return fail(OMAP_ERR_INVALID_ARG, "len/offsets pointer is NULL");
    if (nt) std::memcpy(len_host, q.len.data(), nt * sizeof(int32_t));
    std::memcpy(offsets_host, q.off.data(), (nt + 1) * sizeof(int64_t));
    if (total) host_copy(cells_host, q.cells_pinned ? q.cells_pinned : q.cells.data(), total * sizeof(int32_t));
    if (info_host) *info_host = q.info;
    if (q.cells_pinned) engine->res_pool.release_now(q.cells_pinned);
    engine->queries.erase(it);
    return OMAP_OK;
    API_GUARD_END
}

omap_status_t omap_engine_destroy(omap_engine_t engine) {
    API_GUARD_BEGIN
    if (!engine) return OMAP_OK;
    (void)hipStreamSynchronize(engine->solver.stream);
    for (auto& kv : engine->queries)
        if (kv.second.occ_pinned) engine->occ_pool.release_now(kv.second.occ_pinned);
    engine->solver.destroy();
    delete engine;
    return OMAP_OK;
    API_GUARD_END
}

// ---- diagnostics -----------------------------------------------------------------

static Solver* solver_of(void* handle, int32_t kind) {
    if (!handle) return nullptr;
    if (kind == 0) return &static_cast<omap_plan_s*>(handle)->solver;
    if (kind == 1) return &static_cast<omap_batch_s*>(handle)->solver;
    if (kind == 2) return &static_cast<omap_engine_s*>(handle)->solver;
    return nullptr;
}

omap_status_t omap_profile_enable(void* handle, int32_t kind, int32_t enable) {
    API_GUARD_BEGIN
    Solver* s = solver_of(handle, kind);
    if (!s) return fail(OMAP_ERR_INVALID_ARG, "bad handle or kind");
    return s->profile(enable != 0);
    API_GUARD_END
}

omap_status_t omap_profile_read(void* handle, int32_t kind, int64_t* launches, double* milliseconds,
                                int64_t* cell_updates) {
    API_GUARD_BEGIN
    Solver* s = solver_of(handle, kind);
    if (!s) return fail(OMAP_ERR_INVALID_ARG, "bad handle or kind");
    return s->profile_read(launches, milliseconds, cell_updates);
    API_GUARD_END
}

omap_status_t omap_selftest(void* stream) {
    API_GUARD_BEGIN
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t* d = nullptr;
    HIP_TRY(hipMalloc(&d, 256 * sizeof(int32_t)));
    std::vector<int32_t> h(256, 0);
    hipError_t e = launch_selftest(d, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, 256 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(OMAP_ERR_HIP, "selftest: %s", hipGetErrorString(e));
    for (int l = 0; l < 64; ++l) {
        const int want_left = l == 0 ? 0 : l - 1 + 100;     // lane without a source reads 0
        const int want_right = l == 63 ? 0 : l + 1 + 100;
        if (h[l] != want_left) return fail(OMAP_ERR_HIP, "lane move from left: lane %d got %d want %d", l, h[l], want_left);
        if (h[64 + l] != want_right)
            return fail(OMAP_ERR_HIP, "lane move from right: lane %d got %d want %d", l, h[64 + l], want_right);
    }
    if (h[128] != 0 || h[129] != 4 || (uint32_t)h[130] != 0x7fffffffu || (uint32_t)h[131] != 0x80000000u ||
        h[132] != 3)
        return fail(OMAP_ERR_HIP, "saturating arithmetic: %d %d %d %d %d", h[128], h[129], h[130], h[131], h[132]);
    return OMAP_OK;
    API_GUARD_END
}

}  // extern "C"
