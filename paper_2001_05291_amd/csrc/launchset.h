// A set of instances prepared for the engine: one device allocation holding
// the descriptors, tile tables, initial lists and per-instance workspaces.
#pragma once

#include <vector>

#include "engine.h"

namespace fs {

// What the caller asks of one instance.
struct InstSpec {
    const int32_t *C = nullptr;
    int64_t ldc = 0;
    int32_t B = 0, M = 0, K = 0, R = 0, T = 0, N = 0, mode = 0;
    uint64_t seed = 0;
    const int32_t *init_host = nullptr;  // K ids on the host, or NULL: rank on the device
    fs_trace_rec *trace = nullptr;
    int32_t *best_out = nullptr;
    int32_t *assign_out = nullptr;
    int32_t *sc_cov = nullptr;
    int64_t *sc_dist = nullptr;
    // heterogeneous fleet (typed = false: homogeneous)
    bool typed = false;
    int32_t K_r = 0;
    const int32_t *base_hel = nullptr;   // device B
    const int32_t *rho = nullptr;        // device M, or NULL
    const int32_t *init_rot = nullptr;   // device K (with init_host), or NULL
    int32_t *best_rot_out = nullptr;     // device K, or NULL
};

struct LaunchSet {
    void *dev = nullptr;
    hipStream_t s = nullptr;
    EngineTables tabs;
    EngineConfig cfg;
    std::vector<InstDesc> descs;     // host copies of the device descriptors
    const Tile *rank_rows = nullptr;
    int nrank_rows = 0;
    int32_t Bmax = 0;
    bool any_rank = false;
    bool any_typed = false;
    fs_score *d_scores = nullptr;
    int32_t *d_errors = nullptr;
    LaunchSet() = default;
    LaunchSet(const LaunchSet &) = delete;
    LaunchSet &operator=(const LaunchSet &) = delete;
    ~LaunchSet();
};

// Validates nothing (callers do); plans, allocates (stream-ordered) and
// uploads.  target_wg: sweep workgroups wanted per instance (mission splits).
fs_status build_launch_set(const std::vector<InstSpec> &specs, int target_wg, LaunchSet &ls,
                           hipStream_t s);

// Picks the fastest plan-preserving sweep variant for this launch set's shape
// (cached per shape; skipped when the sweep variant is fixed by environment).
// Needs the initial state (engine_init) in place.
fs_status tune_sweep(LaunchSet &ls, hipStream_t s);

// Reset, ranking, initial state, then N iterations (each: sweep, then
// refresh, which applies the chosen move and recomputes the state).
fs_status run_launch_set(LaunchSet &ls, int32_t N, hipStream_t s);

// Outputs kernel, then scores and error iterations to the host (synchronises).
fs_status collect_results(LaunchSet &ls, std::vector<fs_score> &scores,
                          std::vector<int32_t> &errors, hipStream_t s);

}  // namespace fs
