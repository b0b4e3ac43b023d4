// Drives the repositioning server from several client threads: test
// infrastructure for the sanitizer builds of the library's host runtime (the
// server's scheduler thread, its queues and tables, the launch sets and the
// error and timing state).  The server's calls take host buffers; the plain
// solves of part 4 take device buffers.
//
//   1. A server with four slots and a budget that holds about two of the
//      eight instances' tables: four client threads each own two instances and
//      submit a chain of warm-started requests (a few missions redrawn each
//      time), polling until every result is in; a fifth thread reads the
//      counters meanwhile.
//   2. A server with one slot and room for every table runs the same chains
//      from one thread: every result must equal the first server's (a
//      request's result depends only on its instance's missions, its warm
//      start and its parameters).
//   3. A third server is closed with requests still waiting and running.
//   4. The same chains through fs_tabu_solve, fs_tabu_solve_noalloc,
//      fs_tabu_solve_batch and fs_fleet_solve with a fleet that every base can
//      hold (tables from fs_build_cost_table, each request warm-started from
//      the served result before it) must give the served results.
//
// Prints one line and exits 0 when every result matches, 1 otherwise.
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "fleetstage.h"

namespace {

constexpr int kInstances = 8;
constexpr int kClients = 4;
constexpr int kChain = 3;  // requests per instance

struct Gen {  // 64-bit LCG: input coordinates only
    uint64_t s;
    double uniform(double lo, double hi)
    {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return lo + (hi - lo) * ((double)(s >> 11) * (1.0 / 9007199254740992.0));
    }
    int32_t below(int32_t n)
    {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (int32_t)((s >> 33) % (uint64_t)n);
    }
};

struct Spec {
    int32_t B, M, K, R;
    std::vector<double> bases, missions;
};

struct Request {
    std::vector<int32_t> ids;
    std::vector<double> pd;
};

struct Result {
    std::vector<int32_t> open;
    fs_score score{};
    fs_status status = FS_OK;
};

void draw_point(Gen &g, double *lat, double *lon)
{
    *lat = g.uniform(43.0, 47.0);
    *lon = g.uniform(-81.0, -75.0);
}

Spec make_instance(int i)
{
    Gen g{0x9e3779b97f4a7c15ull * (uint64_t)(i + 1)};
    Spec s;
    s.B = 60 + 20 * i;
    s.M = 800 + 150 * i;
    s.K = 3 + i % 5;
    s.R = 250000 + 10000 * i;
    s.bases.resize(2 * (size_t)s.B);
    s.missions.resize(4 * (size_t)s.M);
    for (int32_t b = 0; b < s.B; ++b) draw_point(g, &s.bases[2 * b], &s.bases[2 * b + 1]);
    for (int32_t m = 0; m < s.M; ++m) {
        draw_point(g, &s.missions[4 * m], &s.missions[4 * m + 1]);
        draw_point(g, &s.missions[4 * m + 2], &s.missions[4 * m + 3]);
    }
    return s;
}

// request r of instance i: n distinct missions get fresh coordinates
Request make_request(const Spec &s, int i, int r)
{
    Gen g{0xd1b54a32d192ed03ull * (uint64_t)(i + 1) + (uint64_t)r};
    Request q;
    const int32_t n = r == 0 ? 0 : 1 + s.M / 20;
    std::vector<char> taken((size_t)s.M, 0);
    while ((int32_t)q.ids.size() < n) {
        const int32_t m = g.below(s.M);
        if (taken[m]) continue;
        taken[m] = 1;
        q.ids.push_back(m);
    }
    q.pd.resize(4 * (size_t)n);
    for (int32_t k = 0; k < n; ++k) {
        draw_point(g, &q.pd[4 * k], &q.pd[4 * k + 1]);
        draw_point(g, &q.pd[4 * k + 2], &q.pd[4 * k + 3]);
    }
    return q;
}

fs_params params_of(int r)
{
    fs_params p{};
    p.tenure = 5;
    p.iterations = 40;
    p.mode = r % 2;  // Tabu and local search alternate along a chain
    return p;
}

bool check(fs_status st, const char *what)
{
    if (st == FS_OK) return true;
    std::fprintf(stderr, "%s: status %d: %s\n", what, (int)st, fs_last_error());
    return false;
}

// waits for one ticket; false on a failed request or call
bool wait_for(fs_server *sv, uint64_t ticket, int32_t K, Result &out)
{
    out.open.assign((size_t)K, -1);
    for (;;) {
        double latency = 0;
        const fs_status st = fs_serve_poll(sv, ticket, out.open.data(), &out.score, &latency);
        if (st == FS_PENDING) {
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            continue;
        }
        out.status = st;
        return check(st, "poll");
    }
}

// every chain of the instances in `mine`, one request in flight per instance
bool run_chains(fs_server *sv, const std::vector<Spec> &specs, const std::vector<int64_t> &ids,
                const std::vector<int> &mine, std::vector<std::vector<Result>> &results)
{
    for (int r = 0; r < kChain; ++r) {
        std::vector<uint64_t> tickets;
        for (int i : mine) {
            const Request q = make_request(specs[i], i, r);
            const fs_params p = params_of(r);
            uint64_t t = 0;
            if (!check(fs_serve_submit(sv, ids[i], q.ids.data(), q.pd.data(),
                                       (int32_t)q.ids.size(), &p, &t),
                       "submit"))
                return false;
            tickets.push_back(t);
        }
        for (size_t k = 0; k < mine.size(); ++k)
            if (!wait_for(sv, tickets[k], specs[mine[k]].K, results[mine[k]][r])) return false;
    }
    return true;
}

bool open_server(int64_t budget, int32_t slots, fs_server **sv)
{
    fs_serve_config cfg{};
    cfg.hbm_budget_bytes = budget;
    cfg.max_slots = slots;
    cfg.device = 0;
    cfg.earth_radius_m = 0;
    cfg.legs = 3;
    return check(fs_serve_open(&cfg, sv), "open");
}

bool register_all(fs_server *sv, const std::vector<Spec> &specs, std::vector<int64_t> &ids)
{
    ids.assign(specs.size(), -1);
    for (size_t i = 0; i < specs.size(); ++i) {
        const Spec &s = specs[i];
        if (!check(fs_serve_register(sv, s.bases.data(), s.B, s.missions.data(), s.M, s.K, s.R,
                                     &ids[i]),
                   "register"))
            return false;
    }
    return true;
}

bool same(const Result &a, const Result &b)
{
    return a.open == b.open && a.score.coverage == b.score.coverage &&
           a.score.distance == b.score.distance && a.score.best_iter == b.score.best_iter;
}

bool hip_ok(hipError_t e, const char *what)
{
    if (e == hipSuccess) return true;
    std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return false;
}

template <typename T>
T *dev_alloc(size_t n, std::vector<void *> &owned)
{
    void *p = nullptr;
    if (!hip_ok(hipMalloc(&p, sizeof(T) * (n ? n : 1)), "hipMalloc")) return nullptr;
    owned.push_back(p);
    return (T *)p;
}

// The served chains again through fs_tabu_solve, fs_tabu_solve_noalloc,
// fs_fleet_solve (no heliport, no rotary-only mission) and one
// fs_tabu_solve_batch per request round over every instance, each warm
// started from the previous request's result like the server.  Counts the
// results that differ from the served ones; -1 on a failed call.
int plain_chains(const std::vector<Spec> &specs, const std::vector<std::vector<Result>> &served)
{
    std::vector<void *> owned;
    struct Dev {
        std::vector<double> missions;
        double *bases = nullptr, *pd = nullptr;
        int32_t *C = nullptr, *init = nullptr, *best = nullptr, *best_na = nullptr,
                *best_b = nullptr;
        int32_t *heli = nullptr, *init_rot = nullptr, *best_f = nullptr, *rot_f = nullptr;
    };
    std::vector<Dev> dv(specs.size());
    for (size_t i = 0; i < specs.size(); ++i) {
        const Spec &s = specs[i];
        Dev &d = dv[i];
        d.missions = s.missions;
        d.bases = dev_alloc<double>(2 * (size_t)s.B, owned);
        d.pd = dev_alloc<double>(4 * (size_t)s.M, owned);
        d.C = dev_alloc<int32_t>((size_t)s.B * s.M, owned);
        d.init = dev_alloc<int32_t>(s.K, owned);
        d.best = dev_alloc<int32_t>(s.K, owned);
        d.best_na = dev_alloc<int32_t>(s.K, owned);
        d.best_b = dev_alloc<int32_t>(s.K, owned);
        d.heli = dev_alloc<int32_t>(s.B, owned);
        d.init_rot = dev_alloc<int32_t>(s.K, owned);
        d.best_f = dev_alloc<int32_t>(s.K, owned);
        d.rot_f = dev_alloc<int32_t>(s.K, owned);
        if (!d.bases || !d.pd || !d.C || !d.init || !d.best || !d.best_na || !d.best_b ||
            !d.heli || !d.init_rot || !d.best_f || !d.rot_f)
            return -1;
        // a fleet with no heliport: the first K/2 slots rotary-wing
        std::vector<int32_t> rot((size_t)s.K);
        for (int32_t k = 0; k < s.K; ++k) rot[k] = k < s.K / 2;
        if (!hip_ok(hipMemset(d.heli, 0, 4 * (size_t)s.B), "clear heliports") ||
            !hip_ok(hipMemcpy(d.init_rot, rot.data(), 4 * (size_t)s.K, hipMemcpyHostToDevice),
                    "copy types"))
            return -1;
        if (!hip_ok(hipMemcpy(d.bases, s.bases.data(), 16 * (size_t)s.B, hipMemcpyHostToDevice),
                    "copy bases"))
            return -1;
    }
    int differ = 0;
    for (int r = 0; r < kChain; ++r) {
        const fs_params p = params_of(r);
        std::vector<fs_instance> batch(specs.size());
        for (size_t i = 0; i < specs.size(); ++i) {
            const Spec &s = specs[i];
            Dev &d = dv[i];
            const Request q = make_request(s, (int)i, r);
            for (size_t k = 0; k < q.ids.size(); ++k)
                std::memcpy(&d.missions[4 * (size_t)q.ids[k]], &q.pd[4 * k], 32);
            if (!hip_ok(hipMemcpy(d.pd, d.missions.data(), 32 * (size_t)s.M,
                                  hipMemcpyHostToDevice),
                        "copy missions") ||
                !check(fs_build_cost_table(d.bases, s.B, d.pd, s.M, 0, 3, d.C, s.M, nullptr,
                                           nullptr),
                       "cost table"))
                return -1;
            const int32_t *init = nullptr;
            if (r > 0) {   // warm start: the previous request's served result
                if (!hip_ok(hipMemcpy(d.init, served[i][r - 1].open.data(), 4 * (size_t)s.K,
                                      hipMemcpyHostToDevice),
                            "copy init"))
                    return -1;
                init = d.init;
            }
            fs_params pr = p;   // the server takes the range from the instance
            pr.range_m = s.R;
            Result a, b;
            if (!check(fs_tabu_solve(d.C, s.M, s.B, s.M, s.K, &pr, init, d.best, &a.score,
                                     nullptr, nullptr, nullptr),
                       "solve") ||
                !check(fs_tabu_solve_noalloc(d.C, s.M, s.B, s.M, s.K, &pr, init, d.best_na,
                                             &b.score, nullptr, nullptr, nullptr),
                       "solve without allocation"))
                return -1;
            a.open.resize(s.K);
            b.open.resize(s.K);
            if (!hip_ok(hipMemcpy(a.open.data(), d.best, 4 * (size_t)s.K, hipMemcpyDeviceToHost),
                        "copy best") ||
                !hip_ok(hipMemcpy(b.open.data(), d.best_na, 4 * (size_t)s.K,
                                  hipMemcpyDeviceToHost),
                        "copy best"))
                return -1;
            if (!same(a, served[i][r])) {
                std::fprintf(stderr, "instance %zu request %d: fs_tabu_solve differs\n", i, r);
                ++differ;
            }
            if (!same(b, served[i][r])) {
                std::fprintf(stderr, "instance %zu request %d: noalloc differs\n", i, r);
                ++differ;
            }
            // with every base an aerodrome and no rotary-only mission, the
            // typed search makes the untyped search's moves
            fs_fleet fl{};
            fl.rotary = s.K / 2;
            fl.fixed = s.K - s.K / 2;
            fl.heliport = d.heli;
            fl.rotary_only = nullptr;
            Result f;
            if (!check(fs_fleet_solve(d.C, s.M, s.B, s.M, &fl, &pr, init,
                                      init ? d.init_rot : nullptr, d.best_f, d.rot_f, &f.score,
                                      nullptr, nullptr, nullptr),
                       "fleet solve"))
                return -1;
            f.open.resize(s.K);
            if (!hip_ok(hipMemcpy(f.open.data(), d.best_f, 4 * (size_t)s.K,
                                  hipMemcpyDeviceToHost),
                        "copy best"))
                return -1;
            if (!same(f, served[i][r])) {
                std::fprintf(stderr, "instance %zu request %d: fleet solve differs\n", i, r);
                ++differ;
            }
            fs_instance &in = batch[i];
            in = fs_instance{};
            in.C = d.C;
            in.ldc = s.M;
            in.B = s.B;
            in.M = s.M;
            in.K = s.K;
            in.range_m = s.R;
            in.init_open = init;
            in.best_open_out = d.best_b;
        }
        std::vector<fs_score> scores(specs.size());
        if (!check(fs_tabu_solve_batch(batch.data(), (int32_t)batch.size(), &p, scores.data(),
                                       nullptr),
                   "batch"))
            return -1;
        for (size_t i = 0; i < specs.size(); ++i) {
            Result c;
            c.score = scores[i];
            c.open.resize(specs[i].K);
            if (!hip_ok(hipMemcpy(c.open.data(), dv[i].best_b, 4 * (size_t)specs[i].K,
                                  hipMemcpyDeviceToHost),
                        "copy best"))
                return -1;
            if (!same(c, served[i][r])) {
                std::fprintf(stderr, "instance %zu request %d: batch differs\n", i, r);
                ++differ;
            }
        }
    }
    for (void *q : owned) (void)hipFree(q);
    return differ;
}

}  // namespace

int main()
{
    std::vector<Spec> specs;
    int64_t table_bytes = 0, largest = 0;
    for (int i = 0; i < kInstances; ++i) {
        specs.push_back(make_instance(i));
        const int64_t t = 4 * (int64_t)specs[i].B * specs[i].M;
        table_bytes += t;
        largest = t > largest ? t : largest;
    }

    // 1. four client threads on a server that must evict
    fs_server *sv = nullptr;
    const int64_t tight = 2 * largest + (1ll << 20);   // about two of the eight tables
    if (!open_server(tight, 4, &sv)) return 1;
    std::vector<int64_t> ids;
    if (!register_all(sv, specs, ids)) return 1;
    std::vector<std::vector<Result>> mixed(kInstances, std::vector<Result>(kChain));
    std::atomic<bool> ok{true}, done{false};
    std::vector<std::thread> clients;
    for (int c = 0; c < kClients; ++c)
        clients.emplace_back([&, c] {
            std::vector<int> mine;
            for (int i = c; i < kInstances; i += kClients) mine.push_back(i);
            if (!run_chains(sv, specs, ids, mine, mixed)) ok = false;
        });
    int64_t polls = 0;
    std::thread watcher([&] {
        while (!done) {
            fs_serve_stats st{};
            if (fs_serve_stats_get(sv, &st) != FS_OK) ok = false;
            ++polls;
            std::this_thread::sleep_for(std::chrono::microseconds(500));
        }
    });
    for (std::thread &t : clients) t.join();
    done = true;
    watcher.join();
    fs_serve_stats stats{};
    if (!check(fs_serve_stats_get(sv, &stats), "stats")) return 1;
    if (!check(fs_serve_close(sv), "close")) return 1;
    if (!ok) return 1;

    // 2. the same chains, one slot, every table resident
    if (!open_server(4 * table_bytes + (64ll << 20), 1, &sv)) return 1;
    if (!register_all(sv, specs, ids)) return 1;
    std::vector<std::vector<Result>> alone(kInstances, std::vector<Result>(kChain));
    for (int i = 0; i < kInstances; ++i)
        if (!run_chains(sv, specs, ids, {i}, alone)) return 1;
    if (!check(fs_serve_close(sv), "close")) return 1;
    int mismatches = 0;
    for (int i = 0; i < kInstances; ++i)
        for (int r = 0; r < kChain; ++r)
            if (!same(mixed[i][r], alone[i][r])) {
                std::fprintf(stderr, "instance %d request %d differs\n", i, r);
                ++mismatches;
            }

    // 3. close with requests waiting and running
    if (!open_server(tight, 2, &sv)) return 1;
    if (!register_all(sv, specs, ids)) return 1;
    for (int i = 0; i < kInstances; ++i) {
        const Request q = make_request(specs[i], i, 1);
        const fs_params p = params_of(0);
        uint64_t t = 0;
        if (!check(fs_serve_submit(sv, ids[i], q.ids.data(), q.pd.data(), (int32_t)q.ids.size(),
                                   &p, &t),
                   "submit"))
            return 1;
    }
    if (!check(fs_serve_close(sv), "close in flight")) return 1;

    // 4. the same chains through the plain, allocation-free and batch solves
    const int plain = plain_chains(specs, mixed);
    if (plain < 0) return 1;
    mismatches += plain;

    std::printf("serve driver: %d requests, %lld evictions, %lld rebuilds, %lld counter reads, "
                "%d mismatches\n",
                kInstances * kChain, (long long)stats.evictions, (long long)stats.rebuilds,
                (long long)polls, mismatches);
    return mismatches == 0 && stats.evictions > 0 ? 0 : 1;
}
