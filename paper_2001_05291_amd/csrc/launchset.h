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

// Device memory a launch set is carved from instead of allocating its own
// (the entry point that allocates nothing): p, cap bytes, 256-byte aligned.
// A launch set built in it uses the dense sweep (the sparse sweep's sorted
// lists are far larger) and the rule-chosen sweep variant (no autotuning,
// which creates events).
struct Workspace {
    void *p = nullptr;
    size_t cap = 0;
};

struct LaunchSet {
    void *dev = nullptr;
    bool owned = true;               // dev was allocated here (freed on destruction)
    bool tune = true;                // the autotuner may time sweep variants
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
// ws: carve the launch set from this workspace instead of allocating
// (FS_E_INVALID when it does not fit).  need: when not NULL, only plan and
// store the device bytes the launch set takes (nothing is allocated,
// uploaded or launched).
fs_status build_launch_set(const std::vector<InstSpec> &specs, int target_wg, LaunchSet &ls,
                           hipStream_t s, const Workspace *ws = nullptr,
                           size_t *need = nullptr);

// Picks the fastest plan-preserving sweep variant for this launch set's shape
// (cached per shape; skipped when the sweep variant is fixed by environment).
// Needs the initial state (engine_init) in place.
fs_status tune_sweep(LaunchSet &ls, hipStream_t s);

// Reset, ranking, initial state, then N iterations (each: sweep, then
// refresh, which applies the chosen move and recomputes the state).
fs_status run_launch_set(LaunchSet &ls, int32_t N, hipStream_t s);

// The single-instance solve behind fs_tabu_solve (ws NULL: device buffers
// allocated stream-ordered) and fs_tabu_solve_noalloc (every device buffer
// carved from ws; FS_E_INVALID before any launch when it does not fit).
fs_status tabu_solve_impl(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                          const fs_params *p, const int32_t *init_open, int32_t *best_open_out,
                          fs_score *score_out, int32_t *assign_out, fs_trace_rec *trace_out,
                          hipStream_t s, const Workspace *ws);

// Outputs kernel, then scores and error iterations to the host (synchronises).
fs_status collect_results(LaunchSet &ls, std::vector<fs_score> &scores,
                          std::vector<int32_t> &errors, hipStream_t s);

}  // namespace fs
