// Single-instance entry points: fs_move_scores and fs_tabu_solve (Section 4.3,
// Algorithm 3, from the base ranking of Section 4.1), driving the engine with
// a launch set of one instance.
#include <algorithm>
#include <cstring>

#include "launchset.h"

namespace fs {
namespace {

struct DeviceBuffer {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~DeviceBuffer()
    {
        if (p) (void)hipFreeAsync(p, s);
    }
};

}  // namespace
}  // namespace fs

// ---------------------------------------------------------------- entry points

extern "C" fs_status fs_move_scores(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                                    const int32_t *open, int32_t K, int32_t range_m,
                                    int32_t *cov_out, int64_t *dist_out, void *stream)
{
    using namespace fs;
    FS_TRY(check_problem(C, ldc, B, M, K, range_m));
    if (!open || !cov_out || !dist_out) return fail(FS_E_INVALID, "NULL open or output pointer");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> ids;
    FS_TRY(fetch_open_list(open, K, B, ids, s));
    FS_TRY(engine_fill_i32(cov_out, (int64_t)K * B, -1, s));
    FS_TRY(engine_fill_i64(dist_out, (int64_t)K * B, -1, s));
    InstSpec sp;
    sp.C = C;
    sp.ldc = ldc;
    sp.B = B;
    sp.M = M;
    sp.K = K;
    sp.R = range_m;
    sp.N = 1;
    sp.init_host = ids.data();
    sp.sc_cov = cov_out;
    sp.sc_dist = dist_out;
    LaunchSet ls;
    FS_TRY(build_launch_set({sp}, env_int("FS_SWEEP_TARGET_WG", 256), ls, s));
    FS_TRY(engine_reset(ls.tabs, ls.Bmax, ls.cfg.Kmax, s));
    FS_TRY(engine_init(ls.tabs, ls.cfg, 0, s));
    if (ls.cfg.sparse) FS_TRY(engine_sparse_prepare(ls.tabs, ls.cfg, s));
    FS_TRY(engine_sweep(ls.tabs, ls.cfg, 1, s));
    FS_HIP(hipStreamSynchronize(s));
    return FS_OK;
}

namespace fs {

fs_status tabu_solve_impl(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                          const fs_params *p, const int32_t *init_open, int32_t *best_open_out,
                          fs_score *score_out, int32_t *assign_out, fs_trace_rec *trace_out,
                          hipStream_t s, const Workspace *ws)
{
    if (!p) return fail(FS_E_INVALID, "params pointer is NULL");
    FS_TRY(check_problem(C, ldc, B, M, K, p->range_m));
    FS_TRY(check_params(p));
    if (!best_open_out || !score_out) return fail(FS_E_INVALID, "NULL output pointer");
    const int target_wg = env_int("FS_SWEEP_TARGET_WG", 256);

    InstSpec sp;
    sp.C = C;
    sp.ldc = ldc;
    sp.B = B;
    sp.M = M;
    sp.K = K;
    sp.R = p->range_m;
    sp.T = p->tenure;
    sp.N = p->iterations;
    sp.mode = p->mode;
    sp.seed = p->seed;
    sp.trace = trace_out;
    sp.best_out = best_open_out;
    sp.assign_out = assign_out;
    const size_t rank_bytes = 8 * (size_t)B + 4 * (size_t)K;
    if (ws) {
        // everything must fit the workspace before anything is launched (the
        // plan does not depend on which bases are open)
        std::vector<int32_t> any(K);
        for (int32_t k = 0; k < K; ++k) any[k] = k;
        sp.init_host = any.data();
        LaunchSet probe;
        size_t need = 0;
        FS_TRY(build_launch_set({sp}, target_wg, probe, s, ws, &need));
        need = std::max(need, init_open ? 0 : rank_bytes);
        if (need > ws->cap)
            return fail(FS_E_INVALID, "B=%d, M=%d, K=%d needs %zu bytes of workspace, more than "
                                      "the %zu available", B, M, K, need, ws->cap);
        sp.init_host = nullptr;
    }

    std::vector<int32_t> init;
    if (init_open) {
        FS_TRY(fetch_open_list(init_open, K, B, init, s));
    } else {
        // base ranking with the grid-wide selection kernel, K ids back to the host
        DeviceBuffer rk;
        rk.s = s;
        if (ws) {
            rk.p = nullptr;
        } else {
            FS_HIP(hipMallocAsync(&rk.p, rank_bytes, s));
        }
        int64_t *sums = (int64_t *)(ws ? ws->p : rk.p);
        int32_t *order = (int32_t *)(sums + B);
        FS_TRY(launch_rank(C, ldc, B, M, K, order, sums, s));
        init.assign(K, 0);
        FS_HIP(hipMemcpyAsync(init.data(), order, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
        FS_HIP(hipStreamSynchronize(s));
        std::sort(init.begin(), init.end());
    }

    sp.init_host = init.data();
    LaunchSet ls;
    FS_TRY(build_launch_set({sp}, target_wg, ls, s, ws));
    FS_TRY(run_launch_set(ls, p->iterations, s));
    std::vector<fs_score> scores;
    std::vector<int32_t> errors;
    FS_TRY(collect_results(ls, scores, errors, s));
    if (errors[0])
        return fail(FS_E_INTERNAL, "refreshed placement value disagrees with the move score at "
                                   "iteration %d", errors[0]);
    *score_out = scores[0];
    return FS_OK;
}

}  // namespace fs

extern "C" fs_status fs_tabu_solve(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                                   const fs_params *p, const int32_t *init_open,
                                   int32_t *best_open_out, fs_score *score_out,
                                   int32_t *assign_out, fs_trace_rec *trace_out, void *stream)
{
    return fs::tabu_solve_impl(C, ldc, B, M, K, p, init_open, best_open_out, score_out,
                               assign_out, trace_out, (hipStream_t)stream, nullptr);
}
