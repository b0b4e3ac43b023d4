// Launch-set construction shared by the single solve, the batch and the
// server.
#include <algorithm>
#include <cstring>

#include "launchset.h"

namespace fs {

LaunchSet::~LaunchSet()
{
    if (dev) (void)hipFreeAsync(dev, s);
}

namespace {
size_t a256(size_t x) { return (x + 255) / 256 * 256; }
}  // namespace

fs_status build_launch_set(const std::vector<InstSpec> &specs, int target_wg, LaunchSet &ls,
                           hipStream_t s)
{
    const int n = (int)specs.size();
    if (n < 1) return fail(FS_E_INVALID, "empty launch set");
    ls.s = s;
    int32_t Kmax = 1, Bmax = 1;
    bool vec4 = true;
    std::vector<int32_t> ncl(n);
    for (int i = 0; i < n; ++i) {
        const InstSpec &p = specs[i];
        ncl[i] = p.B - p.K;
        Kmax = std::max(Kmax, p.K);
        Bmax = std::max(Bmax, p.B);
        vec4 = vec4 && (p.ldc % 4 == 0) && ((uintptr_t)p.C % 16 == 0);
    }
    std::vector<int32_t> sorted_ncl = ncl;
    std::sort(sorted_ncl.begin(), sorted_ncl.end());
    EngineConfig &cfg = ls.cfg;
    cfg.J = choose_rows_per_group(sorted_ncl[n / 2], Kmax);
    cfg.U = choose_unroll(cfg.J);
    cfg.vec4 = vec4;
    // non-temporal row loads once the tables outgrow what the 256 MB
    // Infinity Cache keeps across iterations
    size_t table_bytes = 0;
    for (const InstSpec &p : specs) table_bytes += (size_t)p.B * p.M * 4;
    cfg.nt = env_int("FS_SWEEP_NT", table_bytes > ((size_t)96 << 20)) != 0;
    cfg.Kmax = Kmax;
    ls.Bmax = Bmax;

    std::vector<InstPlan> plans(n);
    std::vector<int32_t> Mp(n);
    for (int i = 0; i < n; ++i) {
        plans[i] = plan_instance(specs[i].B, specs[i].M, specs[i].K, cfg.J, target_wg);
        Mp[i] = (specs[i].M + 3) / 4 * 4;
    }
    std::vector<Tile> sweep, score, refresh, rank_rows;
    build_tiles(plans, Mp, sweep, score, refresh);
    size_t list_ints = 0;
    for (int i = 0; i < n; ++i) {
        if (specs[i].init_host) {
            list_ints += (size_t)specs[i].K + std::max(specs[i].B - specs[i].K, 1);
        } else {
            ls.any_rank = true;
            for (int32_t b = 0; b < specs[i].B; ++b) rank_rows.push_back(Tile{i, b, 0, 0});
        }
    }

    // header: descriptors, tiles, results, initial lists; then workspaces
    const size_t o_desc = 0;
    const size_t o_sweep = o_desc + a256(sizeof(InstDesc) * n);
    const size_t o_score = o_sweep + a256(sizeof(Tile) * sweep.size());
    const size_t o_refresh = o_score + a256(sizeof(Tile) * std::max<size_t>(score.size(), 1));
    const size_t o_rank = o_refresh + a256(sizeof(Tile) * refresh.size());
    const size_t o_scores = o_rank + a256(sizeof(Tile) * std::max<size_t>(rank_rows.size(), 1));
    const size_t o_errors = o_scores + a256(sizeof(fs_score) * n);
    const size_t o_lists = o_errors + a256(sizeof(int32_t) * n);
    const size_t o_ws = o_lists + a256(4 * std::max<size_t>(list_ints, 1));
    std::vector<size_t> ws_off(n);
    size_t total = o_ws;
    for (int i = 0; i < n; ++i) {
        ws_off[i] = total;
        total += instance_bytes(specs[i].B, specs[i].M, specs[i].K, plans[i]);
        if (!specs[i].init_host) total += a256(8 * (size_t)specs[i].B);
    }
    FS_HIP(hipMallocAsync(&ls.dev, total, s));
    char *base = (char *)ls.dev;

    std::vector<char> head(o_ws, 0);
    int32_t *lists_host = (int32_t *)(head.data() + o_lists);
    int32_t *lists_dev = (int32_t *)(base + o_lists);
    size_t lpos = 0;
    ls.descs.assign(n, InstDesc{});
    for (int i = 0; i < n; ++i) {
        const InstSpec &p = specs[i];
        InstDesc &d = ls.descs[i];
        carve_instance(d, base + ws_off[i], p.B, p.M, p.K, plans[i]);
        d.C = p.C;
        d.ldc = p.ldc;
        d.R = p.R;
        d.T = p.T;
        d.N = p.N;
        d.mode = p.mode;
        d.active = 1;
        d.start_step = 0;
        d.trace = p.trace;
        d.sc_cov = p.sc_cov;
        d.sc_dist = p.sc_dist;
        d.best_out = p.best_out;
        d.assign_out = p.assign_out;
        if (p.init_host) {
            d.need_rank = 0;
            d.sums = nullptr;
            // lists of S_1 (parity 1): open list as given, closed list = the
            // complement in ascending id order
            d.open[1] = lists_dev + lpos;
            memcpy(lists_host + lpos, p.init_host, 4 * (size_t)p.K);
            lpos += p.K;
            d.closed[1] = lists_dev + lpos;
            std::vector<unsigned char> in(p.B, 0);
            for (int32_t k = 0; k < p.K; ++k) in[p.init_host[k]] = 1;
            size_t c = 0;
            for (int32_t b = 0; b < p.B; ++b)
                if (!in[b]) lists_host[lpos + c++] = b;
            lpos += std::max(p.B - p.K, 1);
        } else {
            d.need_rank = 1;
            d.sums = (int64_t *)(base + ws_off[i] + instance_bytes(p.B, p.M, p.K, plans[i]));
        }
    }
    memcpy(head.data() + o_desc, ls.descs.data(), sizeof(InstDesc) * n);
    memcpy(head.data() + o_sweep, sweep.data(), sizeof(Tile) * sweep.size());
    if (!score.empty()) memcpy(head.data() + o_score, score.data(), sizeof(Tile) * score.size());
    memcpy(head.data() + o_refresh, refresh.data(), sizeof(Tile) * refresh.size());
    if (!rank_rows.empty())
        memcpy(head.data() + o_rank, rank_rows.data(), sizeof(Tile) * rank_rows.size());
    FS_HIP(hipMemcpyAsync(base, head.data(), head.size(), hipMemcpyHostToDevice, s));
    // the host image is pageable and local: finish the copy before it goes
    FS_HIP(hipStreamSynchronize(s));

    EngineTables &t = ls.tabs;
    t.desc = (const InstDesc *)(base + o_desc);
    t.ninst = n;
    t.sweep = (const Tile *)(base + o_sweep);
    t.nsweep = (int)sweep.size();
    t.score = (const Tile *)(base + o_score);
    t.nscore = (int)score.size();
    t.refresh = (const Tile *)(base + o_refresh);
    t.nrefresh = (int)refresh.size();
    ls.rank_rows = (const Tile *)(base + o_rank);
    ls.nrank_rows = (int)rank_rows.size();
    ls.d_scores = (fs_score *)(base + o_scores);
    ls.d_errors = (int32_t *)(base + o_errors);
    return FS_OK;
}

fs_status run_launch_set(LaunchSet &ls, int32_t N, hipStream_t s)
{
    FS_TRY(engine_reset(ls.tabs, ls.Bmax, ls.cfg.Kmax, s));
    if (ls.any_rank) FS_TRY(engine_rank_lists(ls.tabs, ls.rank_rows, ls.nrank_rows, ls.Bmax, s));
    FS_TRY(engine_init(ls.tabs, ls.cfg, 0, s));
    for (int32_t t = 1; t <= N; ++t) {
        FS_TRY(engine_sweep(ls.tabs, ls.cfg, t, s));
        FS_TRY(engine_refresh(ls.tabs, ls.cfg, t, s));
    }
    return FS_OK;
}

fs_status collect_results(LaunchSet &ls, std::vector<fs_score> &scores,
                          std::vector<int32_t> &errors, hipStream_t s)
{
    const int n = ls.tabs.ninst;
    FS_TRY(engine_outputs(ls.tabs, ls.cfg, ls.d_scores, ls.d_errors, s));
    scores.assign(n, fs_score{});
    errors.assign(n, 0);
    FS_HIP(hipMemcpyAsync(scores.data(), ls.d_scores, sizeof(fs_score) * n, hipMemcpyDeviceToHost, s));
    FS_HIP(hipMemcpyAsync(errors.data(), ls.d_errors, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    return FS_OK;
}

}  // namespace fs
