// Heterogeneous-fleet entry points: fs_fleet_move_scores and fs_fleet_solve
// (Section 3, Eq. 4-10: rotary-wing and fixed-wing vehicles, aerodromes and
// heliports, rotary-only missions; the typed base ranking, the helipad-quota
// part of Algorithm 1; the Tabu search of Section 4.3 over vehicle
// relocations).
// They drive the same engine as the homogeneous calls: a typed instance
// differs only in its per-slot vehicle types, the base kinds carried beside
// the lists and the per-mission kind carried in the nearest-slot word.
#include <algorithm>
#include <vector>

#include "launchset.h"

namespace fs {
namespace {

// Validates the fleet against the bases (host copy of the heliport flags):
// every count non-negative, at least one vehicle, enough aerodromes for the
// fixed-wing vehicles and enough usable bases for all of them.
fs_status check_fleet(const fs_fleet *f, int32_t B, std::vector<int32_t> &hel, hipStream_t s)
{
    if (!f) return fail(FS_E_INVALID, "fleet pointer is NULL");
    if (f->rotary < 0 || f->fixed < 0)
        return fail(FS_E_INVALID, "vehicle counts must be >= 0 (rotary %d, fixed %d)", f->rotary,
                    f->fixed);
    if (!f->heliport) return fail(FS_E_INVALID, "heliport flags pointer is NULL");
    hel.assign(B, 0);
    FS_HIP(hipMemcpyAsync(hel.data(), f->heliport, 4 * (size_t)B, hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    int64_t aero = 0;
    for (int32_t b = 0; b < B; ++b) aero += hel[b] == 0;
    const int64_t heli = B - aero;
    if (aero < f->fixed)
        return fail(FS_E_INVALID, "%lld aerodromes cannot hold %d fixed-wing vehicles",
                    (long long)aero, f->fixed);
    if (aero + std::min<int64_t>(heli, f->rotary) < (int64_t)f->rotary + f->fixed)
        return fail(FS_E_INVALID, "the bases cannot hold %d rotary-wing and %d fixed-wing vehicles",
                    f->rotary, f->fixed);
    return FS_OK;
}

// A given typed placement: K distinct bases with their vehicle types, exactly
// `rotary` rotary-wing ones, no fixed-wing vehicle on a heliport.
fs_status fetch_typed_placement(const int32_t *open, const int32_t *rot, const fs_fleet *f,
                                int32_t B, const std::vector<int32_t> &hel,
                                std::vector<int32_t> &ids, hipStream_t s)
{
    const int32_t K = f->rotary + f->fixed;
    if (!rot) return fail(FS_E_INVALID, "a given placement needs its vehicle types");
    FS_TRY(fetch_open_list(open, K, B, ids, s));
    std::vector<int32_t> types(K, 0);
    FS_HIP(hipMemcpyAsync(types.data(), rot, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    int32_t nrot = 0;
    for (int32_t k = 0; k < K; ++k) {
        nrot += types[k] != 0;
        if (!types[k] && hel[ids[k]])
            return fail(FS_E_INVALID, "slot %d: a fixed-wing vehicle on heliport %d", k, ids[k]);
    }
    if (nrot != f->rotary)
        return fail(FS_E_INVALID, "placement has %d rotary-wing vehicles, the fleet %d", nrot,
                    f->rotary);
    return FS_OK;
}

InstSpec typed_spec(const int32_t *C, int64_t ldc, int32_t B, int32_t M, const fs_fleet *f)
{
    InstSpec sp;
    sp.C = C;
    sp.ldc = ldc;
    sp.B = B;
    sp.M = M;
    sp.K = f->rotary + f->fixed;
    sp.typed = true;
    sp.K_r = f->rotary;
    sp.base_hel = f->heliport;
    sp.rho = f->rotary_only;
    return sp;
}

}  // namespace
}  // namespace fs

extern "C" fs_status fs_fleet_move_scores(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                                          const fs_fleet *fleet, const int32_t *open,
                                          const int32_t *rotary, int32_t range_m,
                                          int32_t *cov_out, int64_t *dist_out, void *stream)
{
    using namespace fs;
    if (!fleet) return fail(FS_E_INVALID, "fleet pointer is NULL");
    const int32_t K = fleet->rotary + fleet->fixed;
    FS_TRY(check_problem(C, ldc, B, M, K, range_m));
    if (!open || !cov_out || !dist_out) return fail(FS_E_INVALID, "NULL open or output pointer");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> hel, ids;
    FS_TRY(check_fleet(fleet, B, hel, s));
    FS_TRY(fetch_typed_placement(open, rotary, fleet, B, hel, ids, s));
    FS_TRY(engine_fill_i32(cov_out, (int64_t)K * B, -1, s));
    FS_TRY(engine_fill_i64(dist_out, (int64_t)K * B, -1, s));
    InstSpec sp = typed_spec(C, ldc, B, M, fleet);
    sp.R = range_m;
    sp.N = 1;
    sp.init_host = ids.data();
    sp.init_rot = rotary;
    sp.sc_cov = cov_out;
    sp.sc_dist = dist_out;
    LaunchSet ls;
    FS_TRY(build_launch_set({sp}, env_int("FS_SWEEP_TARGET_WG", 256), ls, s));
    FS_TRY(engine_reset(ls.tabs, ls.Bmax, ls.cfg.Kmax, s));
    FS_TRY(engine_fleet_lists(ls.tabs, s));
    FS_TRY(engine_init(ls.tabs, ls.cfg, 0, s));
    FS_TRY(engine_sweep(ls.tabs, ls.cfg, 1, s));
    FS_HIP(hipStreamSynchronize(s));
    return FS_OK;
}

extern "C" fs_status fs_fleet_solve(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                                    const fs_fleet *fleet, const fs_params *p,
                                    const int32_t *init_open, const int32_t *init_rotary,
                                    int32_t *best_open_out, int32_t *best_rotary_out,
                                    fs_score *score_out, int32_t *assign_out,
                                    fs_trace_rec *trace_out, void *stream)
{
    using namespace fs;
    if (!p) return fail(FS_E_INVALID, "params pointer is NULL");
    if (!fleet) return fail(FS_E_INVALID, "fleet pointer is NULL");
    const int32_t K = fleet->rotary + fleet->fixed;
    FS_TRY(check_problem(C, ldc, B, M, K, p->range_m));
    FS_TRY(check_params(p));
    if (p->mode > 1)
        return fail(FS_E_INVALID, "typed fleets run modes 0 and 1 (mode %d requested)", p->mode);
    if (!best_open_out || !best_rotary_out || !score_out)
        return fail(FS_E_INVALID, "NULL output pointer");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> hel, ids;
    FS_TRY(check_fleet(fleet, B, hel, s));
    if (init_open) FS_TRY(fetch_typed_placement(init_open, init_rotary, fleet, B, hel, ids, s));

    InstSpec sp = typed_spec(C, ldc, B, M, fleet);
    sp.R = p->range_m;
    sp.T = p->tenure;
    sp.N = p->iterations;
    sp.mode = p->mode;
    sp.seed = p->seed;
    sp.init_host = init_open ? ids.data() : nullptr;   // NULL: typed ranking on the device
    sp.init_rot = init_open ? init_rotary : nullptr;
    sp.trace = trace_out;
    sp.best_out = best_open_out;
    sp.best_rot_out = best_rotary_out;
    sp.assign_out = assign_out;
    LaunchSet ls;
    FS_TRY(build_launch_set({sp}, env_int("FS_SWEEP_TARGET_WG", 256), ls, s));
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
