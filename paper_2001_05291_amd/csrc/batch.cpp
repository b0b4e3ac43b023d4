// fs_tabu_solve_batch: many independent instances of uneven size (Section 4.3,
// Algorithm 3, each from its own base ranking) in one launch set.  Every
// kernel of an iteration spans all instances through the engine's tile
// tables, so the GPU stays full although most instances are small.
#include <algorithm>

#include "launchset.h"

extern "C" fs_status fs_tabu_solve_batch(const fs_instance *inst, int32_t n, const fs_params *p,
                                         fs_score *scores_out, void *stream)
{
    using namespace fs;
    if (!inst || !scores_out) return fail(FS_E_INVALID, "NULL instance or score array");
    if (n < 1) return fail(FS_E_INVALID, "n=%d: need at least one instance", n);
    FS_TRY(check_params(p));
    for (int32_t i = 0; i < n; ++i) {
        const fs_instance &q = inst[i];
        fs_status st = check_problem(q.C, q.ldc, q.B, q.M, q.K, q.range_m);
        if (st == FS_OK && q.B > 32768) st = fail(FS_E_INVALID, "B=%d exceeds 32768", q.B);
        if (st == FS_OK && !q.best_open_out) st = fail(FS_E_INVALID, "best_open_out is NULL");
        if (st != FS_OK) return prefix_error(st, "instance", i);
    }
    hipStream_t s = (hipStream_t)stream;

    // caller-given initial placements: one copy each, one wait, then validation
    std::vector<std::vector<int32_t>> inits(n);
    bool any_init = false;
    for (int32_t i = 0; i < n; ++i) {
        if (!inst[i].init_open) continue;
        any_init = true;
        inits[i].assign(inst[i].K, 0);
        FS_HIP(hipMemcpyAsync(inits[i].data(), inst[i].init_open, 4 * (size_t)inst[i].K,
                              hipMemcpyDeviceToHost, s));
    }
    if (any_init) {
        FS_HIP(hipStreamSynchronize(s));
        for (int32_t i = 0; i < n; ++i)
            if (inst[i].init_open) {
                const fs_status st = check_open_list(inits[i], inst[i].B);
                if (st != FS_OK) return prefix_error(st, "instance", i);
            }
    }

    std::vector<InstSpec> specs(n);
    for (int32_t i = 0; i < n; ++i) {
        const fs_instance &q = inst[i];
        InstSpec &sp = specs[i];
        sp.C = q.C;
        sp.ldc = q.ldc;
        sp.B = q.B;
        sp.M = q.M;
        sp.K = q.K;
        sp.R = q.range_m;
        sp.T = p->tenure;
        sp.N = p->iterations;
        sp.mode = p->mode;
        sp.seed = q.seed;
        sp.init_host = q.init_open ? inits[i].data() : nullptr;
        sp.trace = q.trace_out;
        sp.best_out = q.best_open_out;
        sp.assign_out = q.assign_out;
    }
    // split an instance's missions only when the batch is too small to fill the GPU
    const int target = std::max(0, env_int("FS_BATCH_TARGET_WG", 256) / n);
    LaunchSet ls;
    FS_TRY(build_launch_set(specs, target, ls, s));
    FS_TRY(run_launch_set(ls, p->iterations, s));
    std::vector<fs_score> scores;
    std::vector<int32_t> errors;
    FS_TRY(collect_results(ls, scores, errors, s));
    for (int32_t i = 0; i < n; ++i)
        if (errors[i])
            return fail(FS_E_INTERNAL, "instance %d: refreshed placement value disagrees with the "
                                       "move score at iteration %d", i, errors[i]);
    std::copy(scores.begin(), scores.end(), scores_out);
    return FS_OK;
}
