// Launch-set construction shared by the single solve, the batch and the
// server.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "launchset.h"

namespace fs {

LaunchSet::~LaunchSet()
{
    if (dev && owned) (void)hipFreeAsync(dev, s);
}

namespace {
size_t a256(size_t x) { return (x + 255) / 256 * 256; }
}  // namespace

fs_status build_launch_set(const std::vector<InstSpec> &specs, int target_wg, LaunchSet &ls,
                           hipStream_t s, const Workspace *ws, size_t *need)
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
    std::vector<int32_t> sorted_ncl = ncl, sorted_m(n);
    for (int i = 0; i < n; ++i) sorted_m[i] = specs[i].M;
    std::sort(sorted_ncl.begin(), sorted_ncl.end());
    std::sort(sorted_m.begin(), sorted_m.end());
    EngineConfig &cfg = ls.cfg;
    int64_t total_rows = 0;
    for (int32_t c : ncl) total_rows += c;
    cfg.J = choose_rows_per_group(sorted_ncl[n / 2], sorted_m[n / 2], total_rows, Kmax);
    cfg.U = choose_unroll(cfg.J);
    cfg.vec4 = vec4;
    // non-temporal row loads once the tables outgrow what the 256 MB
    // Infinity Cache keeps across iterations
    size_t table_bytes = 0;
    for (const InstSpec &p : specs) table_bytes += (size_t)p.B * p.M * 4;
    cfg.nt = env_int("FS_SWEEP_NT", table_bytes > ((size_t)96 << 20)) != 0;
    cfg.queue = env_int("FS_SWEEP_QUEUE", 1) != 0;
    cfg.Kmax = Kmax;
    cfg.typed = false;
    for (const InstSpec &p : specs) cfg.typed = cfg.typed || p.typed;
    if (cfg.typed) cfg.U = 1;   // typed sweeps keep one load in flight
    // 16-row groups: untyped in-place vector sweeps with one load in flight
    // (four rows per pass)
    if (cfg.J == 16 && (cfg.typed || !vec4)) cfg.J = 8;
    if (cfg.J == 16) {
        cfg.queue = false;
        cfg.U = 1;
    }
    ls.Bmax = Bmax;
    // the sparse sweep: one homogeneous instance with closed bases and
    // K <= kSparseMaxK (its bins for a block of bases sit in LDS); by default
    // for many closed bases and a long search, where the per-iteration saving
    // (measured 280 -> 158 us at 3,936 closed rows x 100,000 missions) repays
    // the one-off list build (4.3 ms there); at 470 closed rows the dense
    // sweep is faster (16.7 against 21 us)
    const bool sparse_ok = n == 1 && !cfg.typed && specs[0].K <= kSparseMaxK &&
                           specs[0].B > specs[0].K;
    const bool sparse_pays = sparse_ok && specs[0].B - specs[0].K >= 2048 && specs[0].N >= 100;
    cfg.sparse = sparse_ok && !ws && env_int("FS_SPARSE", sparse_pays ? 1 : 0) != 0;

    std::vector<InstPlan> plans(n);
    std::vector<int32_t> Mp(n);
    for (int i = 0; i < n; ++i) {
        plans[i] = cfg.sparse
                       ? plan_sparse(specs[i].B, specs[i].M, specs[i].K, std::max(target_wg, 512))
                       : plan_instance(specs[i].B, specs[i].M, specs[i].K, cfg.J, target_wg);
        Mp[i] = (specs[i].M + 3) / 4 * 4;
    }
    std::vector<Tile> sweep, score, refresh, rank_rows;
    // small K over many missions: a thread per mission scanning every open
    // slot gives a quarter of the refresh workgroups (each re-derives the
    // move, so fewer of them is cheaper)
    int64_t refresh64 = 0;
    for (int i = 0; i < n; ++i) refresh64 += (Mp[i] + kRefreshMissions - 1) / kRefreshMissions;
    cfg.refresh_mpt = env_int("FS_REFRESH_WIDE", Kmax <= 32 && refresh64 >= 4096) != 0
                          ? kBlock : kRefreshMissions;
    // larger K over many missions: 256 missions per 1024-thread workgroup
    // (four waves per 64 missions splitting the slots), a quarter of the
    // workgroups, each reducing the row-group candidates once
    cfg.refresh_wide = cfg.refresh_mpt == kRefreshMissions &&
                       env_int("FS_REFRESH_SPLIT4", refresh64 >= 1024) != 0;
    if (cfg.refresh_wide) cfg.refresh_mpt = kBlock;
    build_tiles(plans, Mp, sweep, score, refresh, cfg.refresh_mpt);
    // few long row groups: 1024-thread workgroups keep four times as many
    // waves in flight, so each thread has fewer dependent load rounds
    std::vector<int32_t> chunks(n);
    for (int i = 0; i < n; ++i) chunks[i] = plans[i].chunk;
    std::sort(chunks.begin(), chunks.end());
    // (forms without a 1024-thread kernel launch 256 threads)
    cfg.wide = env_int("FS_SWEEP_WIDE", cfg.J <= 2 && sweep.size() < 1024 &&
                                            chunks[n / 2] >= 8192) != 0;
    // the persistent search (one workgroup per instance for the whole loop):
    // homogeneous instances of modes 0 and 1 with 16-byte rows whose state fits
    // LDS with two workgroups per CU; the default for a large batch or small
    // instances (where one launch per iteration is mostly launch overhead)
    // (measured: a whole 200-iteration search of a 400 x 5,000 instance in one
    // workgroup is slower than the ragged batch's per-iteration launches, so
    // the persistent search is the default for small instances only, whose
    // tables it stages in LDS when they fit)
    {
        bool can = !cfg.typed && !cfg.sparse && vec4;
        size_t lds = 0, lds_tab = 0;
        int64_t work_max = 0;
        for (int i = 0; i < n && can; ++i) {
            const InstSpec &p = specs[i];
            can = p.mode <= 1 && p.K <= kSoloMaxKPersist && !p.sc_cov && p.M < kSoloMaxMissions;
            lds = std::max(lds, solo_lds_of(Mp[i], p.K, p.B - p.K));
            lds_tab = std::max(lds_tab, solo_lds_of(Mp[i], p.K, p.B - p.K, p.B));
            work_max = std::max(work_max, (int64_t)(p.B - p.K) * Mp[i]);
        }
        can = can && lds + 1024 <= (size_t)80 * 1024;
        const bool pays = work_max <= ((int64_t)1 << 16);
        cfg.persistent = can && env_int("FS_PERSIST", pays ? 1 : 0) != 0;
        cfg.solo_tab = cfg.persistent && lds_tab + 1024 <= (size_t)160 * 1024 &&
                       env_int("FS_PERSIST_TAB", 1) != 0;
        cfg.solo_lds = (uint32_t)(cfg.solo_tab ? lds_tab : lds);
    }
    // the sparse sweep's block scoring fused with the refresh (one instance
    // with mission chunks; not for the full score table, which the sweep
    // launch alone must produce).  Off by default: measured 38.8 us per fused
    // launch against 10.9 + 12.9 us for the two launches at 3,936 closed rows
    // x 100,000 missions (the release fences of 252 scoring workgroups and the
    // waiting refresh workgroups cost more than the launch they save).
    cfg.fuse_score = cfg.sparse && n == 1 && plans[0].nsplit > 1 && !specs[0].sc_cov &&
                     env_int("FS_FUSE", 0) != 0;
    std::vector<Tile> solo;
    if (cfg.persistent) {
        // largest instances first, so that they do not finish last
        std::vector<int> ord(n);
        for (int i = 0; i < n; ++i) ord[i] = i;
        auto work = [&](int i) { return ((int64_t)specs[i].B) * Mp[i]; };
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return work(a) > work(b); });
        for (int i : ord) solo.push_back(Tile{i, 0, 0, 0});
    }
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
    const size_t o_solo = o_rank + a256(sizeof(Tile) * std::max<size_t>(rank_rows.size(), 1));
    const size_t o_scores = o_solo + a256(sizeof(Tile) * std::max<size_t>(solo.size(), 1));
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
    if (need) {
        *need = total;
        return FS_OK;
    }
    if (ws) {
        if (total > ws->cap)
            return fail(FS_E_INVALID, "the solve needs %zu bytes of workspace, more than the "
                                      "%zu bytes available", total, ws->cap);
        ls.dev = ws->p;
        ls.owned = false;
        ls.tune = false;
    } else {
        FS_HIP(hipMallocAsync(&ls.dev, total, s));
    }
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
        d.seed = p.seed;
        d.active = 1;
        d.start_step = 0;
        d.trace = p.trace;
        d.sc_cov = p.sc_cov;
        d.sc_dist = p.sc_dist;
        d.best_out = p.best_out;
        d.assign_out = p.assign_out;
        d.typed = p.typed ? 1 : 0;
        d.K_r = p.typed ? p.K_r : p.K;
        d.base_hel = p.base_hel;
        d.rho = p.rho;
        d.init_rot = p.init_rot;
        d.best_rot_out = p.best_rot_out;
        ls.any_typed = ls.any_typed || p.typed;
        if (p.init_host) {
            d.need_rank = 0;
            d.sums = nullptr;
            // lists of S_1 (parity 1): open list as given, closed list = the
            // complement in ascending id order
            d.open = lists_dev + lpos;
            memcpy(lists_host + lpos, p.init_host, 4 * (size_t)p.K);
            lpos += p.K;
            d.closed = lists_dev + lpos;
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
    if (!solo.empty()) memcpy(head.data() + o_solo, solo.data(), sizeof(Tile) * solo.size());
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
    t.single = n == 1;
    t.solo = (const Tile *)(base + o_solo);
    t.nsolo = (int)solo.size();
    ls.rank_rows = (const Tile *)(base + o_rank);
    ls.nrank_rows = (int)rank_rows.size();
    ls.d_scores = (fs_score *)(base + o_scores);
    ls.d_errors = (int32_t *)(base + o_errors);
    return FS_OK;
}

namespace {

// Shape of a launch set as far as the sweep's speed is concerned.
struct TuneKey {
    int64_t ninst, nsweep, nscore, rows, missions;
    int32_t J, Kmax, vec4, nt, typed;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(ninst, nsweep, nscore, rows, missions, J, Kmax, vec4, nt, typed) <
               std::tie(o.ninst, o.nsweep, o.nscore, o.rows, o.missions, o.J, o.Kmax, o.vec4,
                        o.nt, o.typed);
    }
};

struct Tuned {
    int U;
    bool queue, wide;
};

std::mutex g_tune_mu;
std::map<TuneKey, Tuned> g_tuned;

bool user_fixed_sweep()
{
    return getenv("FS_SWEEP_U") || getenv("FS_SWEEP_QUEUE") || getenv("FS_SWEEP_WIDE");
}

}  // namespace

// Sweep variants that leave the plan (and therefore the workspace) as it is:
// loads in flight per thread, queued scoring, 1024-thread workgroups.  Each is
// timed on the sweep of iteration 1, which may run any number of times: it
// only writes its row groups' candidates (and split partials) and clears the
// accumulators the next refresh fills.  All variants give identical results.
// The fastest is kept for this shape for the rest of the process.
fs_status tune_sweep(LaunchSet &ls, hipStream_t s)
{
    if (!ls.tune || !ls.cfg.vec4 || ls.cfg.sparse || ls.tabs.nsweep == 0 || user_fixed_sweep() ||
        env_int("FS_AUTOTUNE", 1) == 0)
        return FS_OK;
    TuneKey key{ls.tabs.ninst, ls.tabs.nsweep, ls.tabs.nscore, 0, 0,
                ls.cfg.J, ls.cfg.Kmax, ls.cfg.vec4, ls.cfg.nt, ls.cfg.typed};
    for (const InstDesc &d : ls.descs) {
        key.rows += d.nclosed;
        key.missions += d.Mp;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            ls.cfg.U = it->second.U;
            ls.cfg.queue = it->second.queue;
            ls.cfg.wide = it->second.wide;
            return FS_OK;
        }
    }
    std::vector<EngineConfig> cands;
    for (int U : {1, 2, 4})
        for (int q = 0; q < 2; ++q)
            for (int w = 0; w < 2; ++w) {
                if (w && ls.cfg.J > 2 && (q || U != 1)) continue;   // no such wide form
                if (ls.cfg.typed && U != 1) continue;                // typed: U = 1 only
                if (ls.cfg.J >= 8 && U != 1) continue;               // U = 1 only
                if (ls.cfg.J == 16 && q) continue;                   // in place only
                EngineConfig c = ls.cfg;
                c.U = U;
                c.queue = q != 0;
                c.wide = w != 0;
                cands.push_back(c);
            }
    // each candidate: one untimed launch, then kReps launches, each stamped
    // by its own dispatch (no marker packets between the launches)
    constexpr int kReps = 2;
    std::vector<hipEvent_t> ev(2 * kReps * cands.size(), nullptr);
    fs_status st = FS_OK;
    for (size_t i = 0; i < ev.size() && st == FS_OK; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) st = fail(FS_E_DEVICE, "autotune: event");
    timing_suppress(true);
    for (size_t i = 0; i < cands.size() && st == FS_OK; ++i) {
        st = engine_sweep(ls.tabs, cands[i], 1, s);
        for (int r = 0; r < kReps && st == FS_OK; ++r) {
            const size_t e = 2 * (kReps * i + r);
            timing_borrow(ev[e], ev[e + 1]);
            st = engine_sweep(ls.tabs, cands[i], 1, s);
            timing_borrow(nullptr, nullptr);
        }
    }
    timing_suppress(false);
    size_t best = 0;
    float best_ms = 0.f;
    if (st == FS_OK && hipStreamSynchronize(s) != hipSuccess)
        st = fail(FS_E_DEVICE, "autotune: synchronize");
    const bool verbose = env_int("FS_AUTOTUNE_LOG", 0) != 0;
    for (size_t i = 0; i < cands.size() && st == FS_OK; ++i) {
        float ms = 0.f;
        for (int r = 0; r < kReps; ++r) {
            const size_t e = 2 * (kReps * i + r);
            float one = 0.f;
            if (hipEventElapsedTime(&one, ev[e], ev[e + 1]) != hipSuccess) {
                st = fail(FS_E_DEVICE, "autotune: elapsed time");
                break;
            }
            ms = r == 0 ? one : std::min(ms, one);
        }
        if (st != FS_OK) break;
        if (verbose)
            fprintf(stderr, "[autotune] J=%d U=%d queue=%d wide=%d: %.1f us per sweep\n",
                    cands[i].J, cands[i].U, (int)cands[i].queue, (int)cands[i].wide,
                    1000.0 * ms);
        if (i == 0 || ms < best_ms) {
            best = i;
            best_ms = ms;
        }
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st != FS_OK) return st;
    ls.cfg = cands[best];
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = Tuned{ls.cfg.U, ls.cfg.queue, ls.cfg.wide};
    return FS_OK;
}

fs_status run_launch_set(LaunchSet &ls, int32_t N, hipStream_t s)
{
    FS_TRY(engine_reset(ls.tabs, ls.Bmax, ls.cfg.Kmax, s));
    if (ls.any_rank) FS_TRY(engine_rank_lists(ls.tabs, ls.rank_rows, ls.nrank_rows, ls.Bmax, s));
    if (ls.any_typed) FS_TRY(engine_fleet_lists(ls.tabs, s));
    FS_TRY(engine_init(ls.tabs, ls.cfg, 0, s));
    if (ls.cfg.sparse && N >= 1) FS_TRY(engine_sparse_prepare(ls.tabs, ls.cfg, s));
    if (ls.cfg.persistent) return N >= 1 ? engine_persistent(ls.tabs, ls.cfg, s) : FS_OK;
    if (N >= 1) FS_TRY(tune_sweep(ls, s));
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
    FS_HIP(hipMemcpyAsync(scores.data(), ls.d_scores, sizeof(fs_score) * n, hipMemcpyDeviceToHost,
                          s));
    FS_HIP(hipMemcpyAsync(errors.data(), ls.d_errors, sizeof(int32_t) * n, hipMemcpyDeviceToHost,
                          s));
    FS_HIP(hipStreamSynchronize(s));
    return FS_OK;
}

}  // namespace fs
