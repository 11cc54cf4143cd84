// Autotuner of the sweep options (include/omap.h, omap_tune): times the
// propagation of a sample workload under each candidate (schedule, layers per
// visit, columns per lane, tile rows), checks that every candidate's activity
// maps and layer counts are identical to those of the first candidate (the
// defaults) -- the update is monotone and bounded by its fixpoint, so every
// tile schedule must reach the same bits, and a difference is a defect, not a
// tuning outcome -- and returns the fastest.  Choices are kept in a text
// cache keyed by device, use and workload shape class.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "omap.h"
#include "omap_internal.h"

namespace {

__global__ void k_count_diff(const int32_t* __restrict__ a, const int32_t* __restrict__ b, int64_t n,
                             unsigned long long* __restrict__ diff) {
    unsigned long long d = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d += a[i] != b[i];
    if (d) atomicAdd(diff, d);
}

struct Candidate {
    omap_options o;
};

std::vector<Candidate> candidates(int32_t use) {
    std::vector<Candidate> out;
    auto add = [&](int sched, int T, int C, int TH) {
        Candidate c;
        std::memset(&c.o, 0, sizeof c.o);
        c.o.schedule = sched;
        c.o.temporal_depth = T;
        c.o.lane_columns = C;
        c.o.tile_rows = TH;
        out.push_back(c);
    };
    add(OMAP_SCHEDULE_DEFAULT, 0, 0, 0);   // the reference: the defaults of this use
    if (use == OMAP_USE_PLAN) {
        const int a[][3] = {{16, 1, 16}, {16, 1, 32}, {12, 1, 12}, {12, 1, 24}, {8, 1, 8}, {8, 1, 16},
                            {16, 2, 16}, {12, 2, 16}, {32, 2, 32}, {16, 4, 32}};
        for (auto& v : a) add(OMAP_SCHEDULE_ACTIVE, v[0], v[1], v[2]);
        const int b[][2] = {{16, 16}, {16, 32}, {8, 16}};
        for (auto& v : b) add(OMAP_SCHEDULE_BITS, v[0], 0, v[1]);
    } else {
        const int b[][2] = {{16, 16}, {16, 32}, {16, 64}, {8, 8}, {8, 16}, {8, 32}};
        for (auto& v : b) add(OMAP_SCHEDULE_BITS, v[0], 0, v[1]);
        const int a[][3] = {{12, 2, 16}, {16, 2, 16}, {12, 2, 32}, {8, 2, 16}, {16, 1, 16}, {16, 4, 32},
                            {24, 2, 24}};
        for (auto& v : a) add(OMAP_SCHEDULE_ACTIVE, v[0], v[1], v[2]);
    }
    return out;
}

// Shape class of a workload: use, number of mazes and median cells per maze
// (both in powers of two), and the device.
std::string shape_key(const omap_maze_desc* m, int32_t n, int32_t use) {
    std::vector<double> cells(n);
    for (int32_t i = 0; i < n; ++i) cells[i] = (double)m[i].height * m[i].width;
    std::nth_element(cells.begin(), cells.begin() + n / 2, cells.end());
    const int nb = (int)std::floor(std::log2((double)n));
    const int cb = (int)std::floor(std::log2(std::max(1.0, cells[n / 2])));
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    std::ostringstream k;
    k << arch << " use" << use << " n2^" << nb << " cells2^" << cb;
    return k.str();
}

std::mutex g_cache_mu;

bool cache_lookup(const std::string& key, omap_options* o) {
    const char* path = std::getenv("OMAP_TUNE_CACHE");
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        // <key> = schedule T C TH launch
        const size_t eq = line.find(" = ");
        if (eq == std::string::npos || line.compare(0, eq, key) != 0 || eq != key.size()) continue;
        std::istringstream v(line.substr(eq + 3));
        omap_options t;
        std::memset(&t, 0, sizeof t);
        if (v >> t.schedule >> t.temporal_depth >> t.lane_columns >> t.tile_rows >> t.round_launch) {
            *o = t;
            found = true;   // the last entry for a key wins
        }
    }
    return found;
}

void cache_store(const std::string& key, const omap_options& o) {
    const char* path = std::getenv("OMAP_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    std::ofstream f(path, std::ios::app);
    f << key << " = " << o.schedule << ' ' << o.temporal_depth << ' ' << o.lane_columns << ' ' << o.tile_rows
      << ' ' << o.round_launch << '\n';
}

// One candidate: create, propagate `reps` times (the fastest is kept), and
// copy every maze's activity map to `maps` (device, concatenated).
struct Run {
    double ms = 0;
    std::vector<int64_t> layers;
};

omap_status_t run_candidate(const omap_maze_desc* m, int32_t n, int32_t use, const omap_options& o,
                            hipStream_t s, int reps, int32_t* maps, Run* out) {
    out->layers.assign(n, -1);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return OMAP_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return OMAP_ERR_HIP;
    }
    omap_status_t st = OMAP_OK;
    double best = 1e30;
    if (use == OMAP_USE_PLAN) {
        omap_plan_t p = nullptr;
        st = omap_plan_create(&p, m[0].height, m[0].width, m[0].occupancy_dev, m[0].sources_host, m[0].n_sources,
                              m[0].targets_host, m[0].n_targets, &o, s);
        for (int r = 0; st == OMAP_OK && r < reps; ++r) {
            (void)hipEventRecord(e0, s);
            st = omap_propagate(p, OMAP_AUTO_LAYERS, nullptr);
            (void)hipEventRecord(e1, s);
            if (st == OMAP_OK && hipEventSynchronize(e1) == hipSuccess) {
                float t = 0;
                (void)hipEventElapsedTime(&t, e0, e1);
                best = std::min(best, (double)t);
            }
        }
        omap_propagate_info info;
        if (st == OMAP_OK) st = omap_propagate(p, OMAP_AUTO_LAYERS, &info);
        if (st == OMAP_OK) out->layers[0] = info.layers;
        if (st == OMAP_OK) st = omap_get_activity(p, maps, m[0].width);
        if (p) (void)omap_plan_destroy(p);
    } else {
        omap_batch_t b = nullptr;
        st = omap_batch_create(&b, m, n, &o, s);
        for (int r = 0; st == OMAP_OK && r < reps; ++r) {
            (void)hipEventRecord(e0, s);
            st = omap_batch_propagate(b, nullptr, nullptr);
            (void)hipEventRecord(e1, s);
            if (st == OMAP_OK && hipEventSynchronize(e1) == hipSuccess) {
                float t = 0;
                (void)hipEventElapsedTime(&t, e0, e1);
                best = std::min(best, (double)t);
            }
        }
        std::vector<omap_propagate_info> infos(n);
        if (st == OMAP_OK) st = omap_batch_propagate(b, nullptr, infos.data());
        int64_t at = 0;
        for (int32_t i = 0; st == OMAP_OK && i < n; ++i) {
            out->layers[i] = infos[i].layers;
            st = omap_batch_get_activity(b, i, maps + at, m[i].width);
            at += (int64_t)m[i].height * m[i].width;
        }
        if (b) (void)omap_batch_destroy(b);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    out->ms = best;
    return st;
}

}  // namespace

extern "C" omap_status_t omap_tune(const omap_maze_desc* mazes, int32_t n_mazes, int32_t use,
                                   omap_tune_result* result, void* stream) {
    if (!mazes || n_mazes < 1 || !result)
        return omap::report_error(OMAP_ERR_INVALID_ARG, "omap_tune: need mazes, n_mazes >= 1 and result");
    if (use != OMAP_USE_PLAN && use != OMAP_USE_BATCH && use != OMAP_USE_ENGINE)
        return omap::report_error(OMAP_ERR_INVALID_ARG, "omap_tune: unknown use");
    if (use == OMAP_USE_PLAN && n_mazes != 1)
        return omap::report_error(OMAP_ERR_INVALID_ARG, "omap_tune: a plan has one maze");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::string key = shape_key(mazes, n_mazes, use);
    std::memset(result, 0, sizeof *result);
    if (cache_lookup(key, &result->options)) {
        result->from_cache = 1;
        return OMAP_OK;
    }
    int64_t cells = 0;
    for (int32_t i = 0; i < n_mazes; ++i) cells += (int64_t)mazes[i].height * mazes[i].width;
    int32_t *ref = nullptr, *cur = nullptr;
    unsigned long long* d_diff = nullptr;
    if (hipMalloc(&ref, sizeof(int32_t) * (size_t)cells) != hipSuccess ||
        hipMalloc(&cur, sizeof(int32_t) * (size_t)cells) != hipSuccess ||
        hipMalloc(&d_diff, sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        if (ref) (void)hipFree(ref);
        if (cur) (void)hipFree(cur);
        return omap::report_error(OMAP_ERR_OUT_OF_MEMORY, "omap_tune: two copies of the sample's activity maps");
    }
    const std::vector<Candidate> cand = candidates(use);
    std::vector<int64_t> ref_layers;
    omap_status_t st = OMAP_OK;
    double best_ms = 1e30;
    omap_options best{};
    int timed = 0;
    for (size_t k = 0; k < cand.size() && st == OMAP_OK; ++k) {
        omap_options resolved;
        // a candidate this use or this build does not offer is skipped
        if (omap_resolve_options(&cand[k].o, &resolved) != OMAP_OK) continue;
        Run run;
        st = run_candidate(mazes, n_mazes, use, cand[k].o, s, 2, k == 0 ? ref : cur, &run);
        if (st != OMAP_OK) break;
        ++timed;
        if (k == 0) {
            ref_layers = run.layers;
            result->default_ms = run.ms;
        } else {
            unsigned long long diff = 0;
            hipError_t e = hipMemsetAsync(d_diff, 0, sizeof diff, s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_count_diff, dim3(1024), dim3(256), 0, s, ref, cur, cells, d_diff);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipMemcpyAsync(&diff, d_diff, sizeof diff, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                st = omap::report_error(OMAP_ERR_HIP, hipGetErrorString(e));
                break;
            }
            if (diff != 0 || run.layers != ref_layers) {
                char msg[256];
                std::snprintf(msg, sizeof msg,
                              "omap_tune: candidate (schedule %d, depth %d, columns %d, rows %d) differs from the "
                              "defaults in %llu cells", cand[k].o.schedule, cand[k].o.temporal_depth,
                              cand[k].o.lane_columns, cand[k].o.tile_rows, diff);
                st = omap::report_error(OMAP_ERR_HIP, msg);
                break;
            }
        }
        if (run.ms < best_ms) {
            best_ms = run.ms;
            best = cand[k].o;
        }
    }
    (void)hipFree(ref);
    (void)hipFree(cur);
    (void)hipFree(d_diff);
    if (st != OMAP_OK) return st;
    result->options = best;
    result->best_ms = best_ms;
    result->candidates = timed;
    cache_store(key, best);
    return OMAP_OK;
}
