// Repositioning server: continuous batching of Tabu re-solves (Section 4.3)
// over device-resident cost tables.  One scheduler thread owns the device
// work: between batched iterations it retires finished requests, admits
// waiting ones into free slots (building or updating their cost tables, warm
// start lists and initial state), then runs one iteration of every running
// request with the engine's two kernels over a tile table spanning all slots.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>

#include "engine.h"

extern "C" fs_status fs_build_cost_table(const double *base_latlon_deg, int32_t B,
                                         const double *mission_pd_deg, int32_t M,
                                         double earth_radius_m, int32_t legs, int32_t *C,
                                         int64_t ldc, double *Cf, void *stream);

namespace fs {
namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2 };

struct Instance;

struct Request {
    uint64_t ticket = 0;
    int64_t inst = 0;
    Instance *I = nullptr;   // set at submission; instances live until close
    std::vector<int32_t> ids;
    std::vector<double> pd;
    fs_params p{};
    Clock::time_point t_submit, t_done;
    int state = kQueued;
    fs_status status = FS_OK;
    std::string err;
    fs_score score{};
    std::vector<int32_t> best;
};

struct Instance {
    int64_t id = 0;
    int32_t B = 0, M = 0, K = 0, R = 0;
    int64_t ldc = 0;
    std::vector<double> bases, missions;  // host copies (missions as last redrawn)
    double *d_bases = nullptr;
    int32_t *C = nullptr;                 // resident table, or nullptr
    size_t table_bytes = 0;               // table + base coordinates on the device
    std::vector<int32_t> last_best;       // warm start of the next request
    uint64_t last_used = 0;
    bool busy = false;                    // a request of this instance is in a slot
    std::deque<Request *> waiting;        // this instance's requests, in order
};

struct Slot {
    Request *req = nullptr;
    Instance *inst = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    InstDesc desc{};
    int32_t J = 1;          // rows per sweep workgroup of this request
    int32_t finish_step = 0;
    bool fresh = false;     // admitted this round: initial state still to compute
    bool draining = false;  // finished: results on their way to the host
    hipEvent_t ev = nullptr;
    fs_score *h_score = nullptr;
    int32_t *h_err = nullptr;
    int32_t *h_best = nullptr;
    int32_t best_cap = 0;
};

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

size_t workspace_of(int32_t B, int32_t M, int32_t K, bool rank)
{
    const InstPlan plan = plan_instance(B, M, K, 1, 0);
    return a256(instance_bytes(B, M, K, plan)) + (rank ? a256(8 * (size_t)B) : 0);
}

size_t table_of(int32_t B, int32_t M)
{
    const size_t ldc = (size_t)(M + 3) / 4 * 4;
    return a256(4 * (size_t)B * ldc) + a256(16 * (size_t)B);
}

}  // namespace

struct Server {
    fs_serve_config cfg{};
    hipStream_t s = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool closing = false;
    bool failed = false;
    std::string fail_msg;
    // registry and requests (under mu)
    std::map<int64_t, std::unique_ptr<Instance>> insts;
    int64_t next_inst = 1;
    uint64_t next_ticket = 1;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
    std::deque<Request *> submitted;
    fs_serve_stats stats{};
    // scheduler-owned
    std::vector<Instance *> known;   // instances that have had requests
    std::vector<Slot> slots;
    std::deque<Request *> pending;
    int32_t step = 0;
    uint64_t lru_clock = 0;
    int64_t used = 0;
    InstDesc *d_desc = nullptr;
    fs_score *d_scores = nullptr;
    int32_t *d_errors = nullptr;
    char *d_arena = nullptr;
    size_t arena_cap = 0, arena_off = 0;
    std::vector<char *> retired_arenas;   // outgrown this round; freed next round
    Tile *d_tiles = nullptr;          // sweep then refresh tiles of the running slots
    size_t tiles_cap = 0;             // in tiles
    char *h_stage[2] = {nullptr, nullptr};
    size_t stage_cap = 0, stage_off = 0;
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_used[2] = {false, false};
    int round = 0;
    bool tiles_dirty = true;
    int64_t retired_ok = 0;
    int64_t fail_nth = 0;             // FS_SERVE_FAIL_NTH (tests): see retire()
    EngineTables tabs;
    EngineConfig ecfg;

    fs_status init();
    void loop();
    fs_status round_once(bool &idle);
    fs_status begin_stage(size_t need);
    fs_status upload(void *dst, const void *src, size_t n);
    fs_status arena_take(size_t n, char **out);
    fs_status admit(Request *r, int slot, bool &admitted);
    fs_status make_resident(Instance &I, size_t need_ws, bool &ok);
    bool evict_one(const Instance *keep);
    fs_status finish_slot(int slot);
    void retire(int slot, fs_status st, const char *msg);
    fs_status rebuild_tables();
    void fail_all(fs_status st, const std::string &msg);
    void release_device();
};

namespace {

// Sizes of one round's host->device uploads are bounded by this staging buffer.
constexpr size_t kStageBytes = 8u << 20;

}  // namespace

fs_status Server::init()
{
    FS_HIP(hipSetDevice(cfg.device));
    FS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    fail_nth = env_int("FS_SERVE_FAIL_NTH", 0);
    slots.assign(cfg.max_slots, Slot{});
    for (Slot &sl : slots) {
        FS_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
        FS_HIP(hipHostMalloc((void **)&sl.h_score, sizeof(fs_score) + 16, hipHostMallocDefault));
        sl.h_err = (int32_t *)((char *)sl.h_score + sizeof(fs_score));
    }
    FS_HIP(hipMalloc((void **)&d_desc, sizeof(InstDesc) * cfg.max_slots));
    FS_HIP(hipMalloc((void **)&d_scores, sizeof(fs_score) * cfg.max_slots));
    FS_HIP(hipMalloc((void **)&d_errors, sizeof(int32_t) * cfg.max_slots));
    std::vector<InstDesc> blank(cfg.max_slots, InstDesc{});
    FS_HIP(hipMemcpy(d_desc, blank.data(), sizeof(InstDesc) * cfg.max_slots,
                     hipMemcpyHostToDevice));
    stage_cap = kStageBytes;
    for (int b = 0; b < 2; ++b) {
        FS_HIP(hipHostMalloc((void **)&h_stage[b], stage_cap, hipHostMallocDefault));
        FS_HIP(hipEventCreateWithFlags(&stage_ev[b], hipEventDisableTiming));
    }
    ecfg.J = 1;
    ecfg.U = 4;
    ecfg.vec4 = true;
    ecfg.nt = false;
    ecfg.Kmax = 1;
    // in-place scoring: measured ahead of the queued form on the repositioning
    // load (saturation 1,543 against 1,530 requests/s, p99 at 0.8x 21.0
    // against 22.3 ms)
    ecfg.queue = env_int("FS_SERVE_QUEUE", 0) != 0;
    tabs.desc = d_desc;
    tabs.ninst = cfg.max_slots;
    return FS_OK;
}

// Staging buffer of this round: wait until the copies that last read it have
// run, then hand out space from its start.
fs_status Server::begin_stage(size_t need)
{
    const int b = round & 1;
    if (stage_used[b]) FS_HIP(hipEventSynchronize(stage_ev[b]));
    stage_used[b] = false;
    stage_off = 0;
    if (need > stage_cap) {
        FS_HIP(hipStreamSynchronize(s));
        for (int q = 0; q < 2; ++q) {
            FS_HIP(hipHostFree(h_stage[q]));
            h_stage[q] = nullptr;
        }
        stage_cap = a256(need);
        for (int q = 0; q < 2; ++q)
            FS_HIP(hipHostMalloc((void **)&h_stage[q], stage_cap, hipHostMallocDefault));
    }
    arena_off = 0;
    // every launch that used an outgrown arena was enqueued last round
    for (char *a : retired_arenas) FS_HIP(hipFreeAsync(a, s));
    retired_arenas.clear();
    return FS_OK;
}

// Stream-ordered copy of n host bytes through the pinned staging buffer.
fs_status Server::upload(void *dst, const void *src, size_t n)
{
    if (n == 0) return FS_OK;
    if (stage_off + n > stage_cap) {
        // this round outgrew the staging buffer: drain and start over
        FS_HIP(hipStreamSynchronize(s));
        stage_off = 0;
        if (n > stage_cap) {
            FS_HIP(hipHostFree(h_stage[round & 1]));
            h_stage[round & 1] = nullptr;
            const size_t cap = a256(n);
            FS_HIP(hipHostMalloc((void **)&h_stage[round & 1], cap, hipHostMallocDefault));
            // keep both buffers at least this large
            const int o = (round + 1) & 1;
            if (stage_used[o]) FS_HIP(hipEventSynchronize(stage_ev[o]));
            stage_used[o] = false;
            FS_HIP(hipHostFree(h_stage[o]));
            h_stage[o] = nullptr;
            FS_HIP(hipHostMalloc((void **)&h_stage[o], cap, hipHostMallocDefault));
            stage_cap = cap;
        }
    }
    char *h = h_stage[round & 1] + stage_off;
    memcpy(h, src, n);
    stage_off += a256(n);
    FS_HIP(hipMemcpyAsync(dst, h, n, hipMemcpyHostToDevice, s));
    stage_used[round & 1] = true;
    return FS_OK;
}

// Device scratch for this round's tile tables (reused every round: the copies
// into it are ordered after the kernels that read it last round).
fs_status Server::arena_take(size_t n, char **out)
{
    n = a256(std::max<size_t>(n, 16));
    if (arena_off + n > arena_cap) {
        const size_t cap = std::max(2 * arena_cap, a256(arena_off + n) + (1u << 20));
        char *fresh = nullptr;
        FS_HIP(hipMallocAsync((void **)&fresh, cap, s));
        // launches of this round may still be enqueued against the old one
        if (d_arena) retired_arenas.push_back(d_arena);
        d_arena = fresh;
        arena_cap = cap;
        arena_off = 0;
    }
    *out = d_arena + arena_off;
    arena_off += n;
    return FS_OK;
}

bool Server::evict_one(const Instance *keep)
{
    Instance *victim = nullptr;
    for (Instance *I : known) {
        if (I == keep || I->busy || !I->C) continue;
        if (!victim || I->last_used < victim->last_used) victim = I;
    }
    if (!victim) return false;
    (void)hipFreeAsync(victim->C, s);
    (void)hipFreeAsync(victim->d_bases, s);
    victim->C = nullptr;
    victim->d_bases = nullptr;
    used -= (int64_t)victim->table_bytes;
    {
        std::lock_guard<std::mutex> lk(mu);
        stats.evictions += 1;
        stats.resident_bytes -= (int64_t)victim->table_bytes;
    }
    return true;
}

// Makes room for the instance's table (if not resident) plus a workspace of
// need_ws bytes, evicting idle tables; builds the table.  ok = false when the
// room cannot be made now.
fs_status Server::make_resident(Instance &I, size_t need_ws, bool &ok)
{
    const size_t need = need_ws + (I.C ? 0 : I.table_bytes);
    while (used + (int64_t)need > cfg.hbm_budget_bytes)
        if (!evict_one(&I)) {
            ok = false;
            return FS_OK;
        }
    ok = true;
    if (I.C) return FS_OK;
    FS_HIP(hipMallocAsync((void **)&I.C, 4 * (size_t)I.B * I.ldc, s));
    FS_HIP(hipMallocAsync((void **)&I.d_bases, 16 * (size_t)I.B, s));
    double *d_m = nullptr;
    FS_HIP(hipMallocAsync((void **)&d_m, 32 * (size_t)I.M, s));
    FS_TRY(upload(I.d_bases, I.bases.data(), 16 * (size_t)I.B));
    FS_TRY(upload(d_m, I.missions.data(), 32 * (size_t)I.M));
    FS_TRY(fs_build_cost_table(I.d_bases, I.B, d_m, I.M, cfg.earth_radius_m, cfg.legs, I.C, I.ldc,
                               nullptr, s));
    FS_HIP(hipFreeAsync(d_m, s));
    used += (int64_t)I.table_bytes;
    std::lock_guard<std::mutex> lk(mu);
    stats.rebuilds += 1;
    stats.resident_bytes += (int64_t)I.table_bytes;
    return FS_OK;
}

// Request r (head of its instance's queue, instance idle) into free slot i:
// redraw its missions, warm start, workspace, descriptor.
fs_status Server::admit(Request *r, int i, bool &admitted)
{
    Instance &I = *r->I;
    const bool rank = I.last_best.empty();
    const size_t ws = workspace_of(I.B, I.M, I.K, rank);
    bool ok = false;
    FS_TRY(make_resident(I, ws, ok));
    if (!ok) {
        admitted = false;
        return FS_OK;
    }
    admitted = true;
    const int32_t n = (int32_t)r->ids.size();
    if (n > 0) {
        char *buf = nullptr;
        FS_HIP(hipMallocAsync((void **)&buf, a256(4 * (size_t)n) + 32 * (size_t)n, s));
        int32_t *d_ids = (int32_t *)buf;
        double *d_pd = (double *)(buf + a256(4 * (size_t)n));
        FS_TRY(upload(d_ids, r->ids.data(), 4 * (size_t)n));
        FS_TRY(upload(d_pd, r->pd.data(), 32 * (size_t)n));
        FS_TRY(launch_cost_columns(I.d_bases, I.B, d_ids, d_pd, n, I.M, cfg.earth_radius_m,
                                   cfg.legs, I.C, I.ldc, s));
        FS_HIP(hipFreeAsync(buf, s));
        for (int32_t q = 0; q < n; ++q)
            memcpy(&I.missions[4 * (size_t)r->ids[q]], &r->pd[4 * (size_t)q], 32);
    }
    Slot &sl = slots[i];
    FS_HIP(hipMallocAsync(&sl.ws, ws, s));
    sl.ws_bytes = ws;
    used += (int64_t)ws;
    // instances with many rows, or short rows, sweep 4 rows per workgroup
    // (fewer re-reads of the per-mission state; enough streaming per
    // workgroup); their tiles are launched as a second class
    const int32_t ncl = I.B - I.K;
    int32_t J = (ncl >= env_int("FS_SERVE_TALL_ROWS", 1024) || (I.M < 8192 && ncl >= 16)) ? 4 : 1;
    if (sweep_lds_of(J, I.K) > ((size_t)56 << 10)) J = 1;
    const InstPlan plan = plan_instance(I.B, I.M, I.K, J, 0);
    InstDesc d{};
    carve_instance(d, (char *)sl.ws, I.B, I.M, I.K, plan);
    d.C = I.C;
    d.ldc = I.ldc;
    d.R = I.R;
    d.T = r->p.tenure;
    d.N = r->p.iterations;
    d.mode = r->p.mode;
    d.seed = r->p.seed;
    d.active = 1;
    d.start_step = step;
    d.need_rank = rank ? 1 : 0;
    d.sums = rank ? (int64_t *)((char *)sl.ws + a256(instance_bytes(I.B, I.M, I.K, plan)))
                  : nullptr;
    if (!rank) {
        std::vector<int32_t> closed;
        std::vector<unsigned char> in(I.B, 0);
        for (int32_t b : I.last_best) in[b] = 1;
        for (int32_t b = 0; b < I.B; ++b)
            if (!in[b]) closed.push_back(b);
        FS_TRY(upload(d.open, I.last_best.data(), 4 * (size_t)I.K));
        if (!closed.empty()) FS_TRY(upload(d.closed, closed.data(), 4 * closed.size()));
    }
    sl.desc = d;
    sl.J = J;
    sl.req = r;
    sl.inst = &I;
    sl.fresh = true;
    sl.draining = false;
    sl.finish_step = step + d.N;
    if (sl.best_cap < I.K) {
        if (sl.h_best) FS_HIP(hipHostFree(sl.h_best));
        FS_HIP(hipHostMalloc((void **)&sl.h_best, 4 * (size_t)I.K, hipHostMallocDefault));
        sl.best_cap = I.K;
    }
    I.busy = true;
    I.last_used = ++lru_clock;
    tiles_dirty = true;
    std::lock_guard<std::mutex> lk(mu);
    r->state = kRunning;
    stats.workspace_bytes += (int64_t)ws;
    stats.running += 1;
    stats.queued -= 1;
    return FS_OK;
}

// Results of a slot whose last iteration has been enqueued: sorted best
// placement, score and consistency check to pinned memory, then an event.
fs_status Server::finish_slot(int i)
{
    Slot &sl = slots[i];
    EngineTables one;
    one.desc = d_desc + i;
    one.ninst = 1;
    FS_TRY(engine_outputs(one, ecfg, d_scores + i, d_errors + i, s));
    FS_HIP(hipMemcpyAsync(sl.h_score, d_scores + i, sizeof(fs_score), hipMemcpyDeviceToHost, s));
    FS_HIP(hipMemcpyAsync(sl.h_err, d_errors + i, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FS_HIP(hipMemcpyAsync(sl.h_best, sl.desc.best_sorted, 4 * (size_t)sl.inst->K,
                          hipMemcpyDeviceToHost, s));
    FS_HIP(hipEventRecord(sl.ev, s));
    sl.draining = true;
    tiles_dirty = true;
    return FS_OK;
}

void Server::retire(int i, fs_status st, const char *msg)
{
    Slot &sl = slots[i];
    Instance &I = *sl.inst;
    Request *r = sl.req;
    std::vector<int32_t> best;
    // (host-side fault injection for tests of this path: the n-th request
    // retired with FS_OK is reported as failing the device-side check)
    if (st == FS_OK && ++retired_ok == fail_nth && *sl.h_err == 0) *sl.h_err = -1;
    if (st == FS_OK) {
        best.assign(sl.h_best, sl.h_best + I.K);
        // only a consistent result seeds the instance's next warm start; after
        // a failed one the next request starts from the last good placement
        // (or the base ranking if there is none)
        if (*sl.h_err == 0) I.last_best = best;
    }
    (void)hipFreeAsync(sl.ws, s);
    used -= (int64_t)sl.ws_bytes;
    I.busy = false;
    I.last_used = ++lru_clock;
    {
        std::lock_guard<std::mutex> lk(mu);
        stats.workspace_bytes -= (int64_t)sl.ws_bytes;
        stats.running -= 1;
        stats.completed += 1;
        r->t_done = Clock::now();
        r->state = kDone;
        r->status = st;
        if (st == FS_OK) {
            r->score = *sl.h_score;
            r->best = std::move(best);
            if (*sl.h_err) {
                r->status = FS_E_INTERNAL;
                r->err = *sl.h_err > 0
                             ? "refreshed placement value disagrees with the move score at "
                               "iteration " + std::to_string(*sl.h_err)
                             : std::string("consistency failure injected by FS_SERVE_FAIL_NTH");
            }
        } else {
            r->err = msg ? msg : "request failed";
        }
    }
    cv.notify_all();
    sl.req = nullptr;
    sl.inst = nullptr;
    sl.ws = nullptr;
    sl.ws_bytes = 0;
    sl.draining = false;
    sl.fresh = false;
    sl.desc = InstDesc{};
    tiles_dirty = true;
}

// Descriptors of every slot and the tile tables of the running ones.
fs_status Server::rebuild_tables()
{
    std::vector<InstDesc> descs(slots.size(), InstDesc{});
    std::vector<Tile> sweep, tall, lng, refresh;
    int32_t Kmax = 1, Kmax_tall = 1, Kmax_long = 1;
    // four-row instances with long rows sweep in 1024-thread workgroups, the
    // others in 256-thread workgroups (short rows would leave most of a wide
    // workgroup idle); measured on the repositioning load: saturation 1,532
    // -> 1,586 requests/s, p99 at 0.8x load 21.8 -> 18.0 ms
    const int32_t long_rows = env_int("FS_SERVE_LONG_ROWS", 8192);
    size_t table_bytes = 0;
    for (size_t i = 0; i < slots.size(); ++i) {
        const Slot &sl = slots[i];
        if (!sl.req) continue;
        descs[i] = sl.desc;
        if (sl.draining) continue;
        const InstDesc &d = sl.desc;
        Kmax = std::max(Kmax, d.K);
        table_bytes += (size_t)d.B * d.M * 4;
        const bool is_long = sl.J == 4 && d.M >= long_rows;
        if (is_long)
            Kmax_long = std::max(Kmax_long, d.K);
        else if (sl.J == 4)
            Kmax_tall = std::max(Kmax_tall, d.K);
        for (int32_t g = 0; g < std::max(d.ngroups, 1); ++g)
            (sl.J == 4 ? (is_long ? lng : tall) : sweep).push_back(Tile{(int32_t)i, g, 0, 0});
        for (int32_t g = 0; g < (d.Mp + kRefreshMissions - 1) / kRefreshMissions; ++g)
            refresh.push_back(Tile{(int32_t)i, g, 0, 0});
    }
    FS_TRY(upload(d_desc, descs.data(), sizeof(InstDesc) * descs.size()));
    // the tables stay until the set of running slots changes; a copy into
    // them is stream-ordered after every kernel that read the old contents
    const size_t ntiles = sweep.size() + tall.size() + lng.size() + refresh.size();
    if (ntiles > tiles_cap) {
        const size_t cap = std::max(ntiles, 2 * tiles_cap);
        Tile *fresh = nullptr;
        FS_HIP(hipMallocAsync((void **)&fresh, sizeof(Tile) * cap, s));
        if (d_tiles) FS_HIP(hipFreeAsync(d_tiles, s));
        d_tiles = fresh;
        tiles_cap = cap;
    }
    const size_t nshort = sweep.size(), ntall = tall.size(), nlong = lng.size();
    sweep.insert(sweep.end(), tall.begin(), tall.end());
    sweep.insert(sweep.end(), lng.begin(), lng.end());
    sweep.insert(sweep.end(), refresh.begin(), refresh.end());
    FS_TRY(upload(d_tiles, sweep.data(), sizeof(Tile) * ntiles));
    tabs.sweep = d_tiles;
    tabs.nsweep = (int)nshort;
    tabs.sweep_tall = d_tiles + nshort;
    tabs.nsweep_tall = (int)ntall;
    tabs.sweep_long = d_tiles + nshort + ntall;
    tabs.nsweep_long = (int)nlong;
    tabs.refresh = d_tiles + nshort + ntall + nlong;
    tabs.nrefresh = (int)refresh.size();
    tabs.score = nullptr;
    tabs.nscore = 0;
    ecfg.Kmax = Kmax;
    ecfg.Kmax_tall = Kmax_tall;
    ecfg.Kmax_long = Kmax_long;
    ecfg.nt = table_bytes > ((size_t)96 << 20);
    tiles_dirty = false;
    return FS_OK;
}

// One scheduler round.  idle = nothing to do until something is submitted.
fs_status Server::round_once(bool &idle)
{
    ++round;
    FS_TRY(begin_stage(0));
    // retire finished slots whose results have arrived
    for (size_t i = 0; i < slots.size(); ++i) {
        Slot &sl = slots[i];
        if (sl.req && sl.draining) {
            const hipError_t e = hipEventQuery(sl.ev);
            if (e == hipSuccess) {
                retire((int)i, FS_OK, nullptr);
            } else if (e != hipErrorNotReady) {
                return fail(FS_E_DEVICE, "request completion: %s", hipGetErrorString(e));
            }
        }
    }
    // admit waiting requests: in submission order, skipping those whose
    // instance is busy or that do not fit yet (no head-of-line blocking)
    for (auto it = pending.begin(); it != pending.end();) {
        int free_slot = -1;
        for (size_t i = 0; i < slots.size(); ++i)
            if (!slots[i].req) {
                free_slot = (int)i;
                break;
            }
        if (free_slot < 0) break;
        Request *r = *it;
        Instance &I = *r->I;
        if (I.busy || I.waiting.front() != r) {
            ++it;
            continue;
        }
        bool admitted = false;
        FS_TRY(admit(r, free_slot, admitted));
        if (!admitted) {
            ++it;
            continue;
        }
        I.waiting.pop_front();
        it = pending.erase(it);
    }
    // descriptors and tiles when the set of slots has changed
    if (tiles_dirty) FS_TRY(rebuild_tables());
    // initial state of the requests admitted this round
    for (size_t i = 0; i < slots.size(); ++i) {
        Slot &sl = slots[i];
        if (!sl.req || !sl.fresh) continue;
        sl.fresh = false;
        const InstDesc &d = sl.desc;
        std::vector<Tile> rt, rows;
        for (int32_t g = 0; g < (d.Mp + kRefreshMissions - 1) / kRefreshMissions; ++g)
            rt.push_back(Tile{0, g, 0, 0});
        if (d.need_rank)
            for (int32_t b = 0; b < d.B; ++b) rows.push_back(Tile{0, b, 0, 0});
        char *p = nullptr;
        FS_TRY(arena_take(sizeof(Tile) * rt.size(), &p));
        FS_TRY(upload(p, rt.data(), sizeof(Tile) * rt.size()));
        EngineTables one;
        one.desc = d_desc + i;
        one.ninst = 1;
        one.refresh = (const Tile *)p;
        one.nrefresh = (int)rt.size();
        EngineConfig c1 = ecfg;
        c1.Kmax = d.K;
        FS_TRY(engine_reset(one, d.B, d.K, s));
        if (d.need_rank) {
            char *q = nullptr;
            FS_TRY(arena_take(sizeof(Tile) * rows.size(), &q));
            FS_TRY(upload(q, rows.data(), sizeof(Tile) * rows.size()));
            FS_TRY(engine_rank_lists(one, (const Tile *)q, (int)rows.size(), d.B, s));
        }
        FS_TRY(engine_init(one, c1, d.start_step, s));
        if (d.N == 0) FS_TRY(finish_slot((int)i));
    }
    // one batched iteration of every running request
    bool running = false;
    for (const Slot &sl : slots)
        if (sl.req && !sl.draining) running = true;
    if (running) {
        if (tiles_dirty) FS_TRY(rebuild_tables());
        ++step;
        FS_TRY(engine_sweep(tabs, ecfg, step, s));
        FS_TRY(engine_refresh(tabs, ecfg, step, s));
        {
            std::lock_guard<std::mutex> lk(mu);
            stats.steps += 1;
        }
        for (size_t i = 0; i < slots.size(); ++i) {
            Slot &sl = slots[i];
            if (sl.req && !sl.draining && sl.finish_step == step) FS_TRY(finish_slot((int)i));
        }
    }
    FS_HIP(hipEventRecord(stage_ev[round & 1], s));
    bool draining = false;
    for (const Slot &sl : slots)
        if (sl.req && sl.draining) draining = true;
    if (!running && draining) {
        // only results in flight: wait for the oldest instead of spinning
        for (Slot &sl : slots)
            if (sl.req && sl.draining) {
                FS_HIP(hipEventSynchronize(sl.ev));
                break;
            }
    }
    idle = !running && !draining;
    return FS_OK;
}

void Server::fail_all(fs_status st, const std::string &msg)
{
    std::lock_guard<std::mutex> lk(mu);
    failed = true;
    fail_msg = msg;
    for (auto &kv : requests) {
        Request *r = kv.second.get();
        if (r->state != kDone) {
            r->state = kDone;
            r->status = st;
            r->err = msg;
            r->t_done = Clock::now();
        }
    }
    cv.notify_all();
}

void Server::loop()
{
    if (hipSetDevice(cfg.device) != hipSuccess) {
        fail_all(FS_E_DEVICE, "scheduler could not select the device");
        return;
    }
    bool idle = true;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return closing || !submitted.empty() || !idle || !pending.empty(); });
            if (closing) break;
            for (Request *r : submitted) {
                if (std::find(known.begin(), known.end(), r->I) == known.end())
                    known.push_back(r->I);
                r->I->waiting.push_back(r);
                pending.push_back(r);
            }
            submitted.clear();
        }
        const fs_status st = round_once(idle);
        if (st != FS_OK) {
            fail_all(st, fs_last_error());
            break;
        }
        if (idle && !pending.empty()) {
            // waiting requests that cannot be admitted while nothing runs
            // will never fit: fail them rather than spin
            bool progress = false;
            for (const Slot &sl : slots)
                if (sl.req) progress = true;
            if (!progress) {
                std::lock_guard<std::mutex> lk(mu);
                for (Request *r : pending) {
                    r->state = kDone;
                    r->status = FS_E_BUDGET;
                    r->err = "request does not fit the device-memory budget";
                    r->t_done = Clock::now();
                    r->I->waiting.clear();
                    stats.queued -= 1;
                }
                pending.clear();
                cv.notify_all();
            }
        }
    }
    (void)hipStreamSynchronize(s);
}

void Server::release_device()
{
    if (s) (void)hipStreamSynchronize(s);
    for (Instance *I : known) {
        if (I->C) (void)hipFreeAsync(I->C, s);
        if (I->d_bases) (void)hipFreeAsync(I->d_bases, s);
        I->C = nullptr;
        I->d_bases = nullptr;
    }
    for (Slot &sl : slots) {
        if (sl.ws) (void)hipFreeAsync(sl.ws, s);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.h_score) (void)hipHostFree(sl.h_score);
        if (sl.h_best) (void)hipHostFree(sl.h_best);
    }
    if (d_arena) (void)hipFreeAsync(d_arena, s);
    for (char *a : retired_arenas) (void)hipFreeAsync(a, s);
    retired_arenas.clear();
    if (d_tiles) (void)hipFreeAsync(d_tiles, s);
    if (s) (void)hipStreamSynchronize(s);
    if (d_desc) (void)hipFree(d_desc);
    if (d_scores) (void)hipFree(d_scores);
    if (d_errors) (void)hipFree(d_errors);
    for (int b = 0; b < 2; ++b) {
        if (h_stage[b]) (void)hipHostFree(h_stage[b]);
        if (stage_ev[b]) (void)hipEventDestroy(stage_ev[b]);
    }
    if (s) (void)hipStreamDestroy(s);
}

}  // namespace fs

struct fs_server {
    fs::Server impl;
};

using fs::fail;

extern "C" fs_status fs_serve_open(const fs_serve_config *cfg, fs_server **out)
{
    if (!cfg || !out) return fail(FS_E_INVALID, "NULL config or output pointer");
    if (cfg->hbm_budget_bytes <= 0) return fail(FS_E_INVALID, "hbm_budget_bytes must be > 0");
    if (cfg->max_slots < 1 || cfg->max_slots > 4096)
        return fail(FS_E_INVALID, "max_slots=%d outside [1, 4096]", cfg->max_slots);
    if (cfg->legs != 2 && cfg->legs != 3) return fail(FS_E_INVALID, "legs must be 2 or 3");
    if (!(cfg->earth_radius_m >= 0.0) || cfg->earth_radius_m > 1.1e8)
        return fail(FS_E_INVALID, "earth radius out of range");
    if (cfg->device < 0) return fail(FS_E_INVALID, "negative device ordinal");
    std::unique_ptr<fs_server> sv(new fs_server);
    sv->impl.cfg = *cfg;
    const fs_status st = sv->impl.init();
    if (st != FS_OK) {
        sv->impl.release_device();
        return st;
    }
    fs::Server *S = &sv->impl;
    S->th = std::thread([S] { S->loop(); });
    *out = sv.release();
    return FS_OK;
}

extern "C" fs_status fs_serve_register(fs_server *sv, const double *base_latlon_deg, int32_t B,
                                       const double *mission_pd_deg, int32_t M, int32_t K,
                                       int32_t range_m, int64_t *instance_id)
{
    using namespace fs;
    if (!sv || !base_latlon_deg || !mission_pd_deg || !instance_id)
        return fail(FS_E_INVALID, "NULL argument");
    if (B < 1 || M < 1) return fail(FS_E_INVALID, "B=%d, M=%d: both must be >= 1", B, M);
    if (B > 32768) return fail(FS_E_INVALID, "B=%d exceeds 32768", B);
    if ((int64_t)M + 3 > INT32_MAX) return fail(FS_E_INVALID, "M=%d too large", M);
    if (K < 1 || K > B || K > kMaxK) return fail(FS_E_INVALID, "K=%d outside [1, min(B, %d)]", K, kMaxK);
    if (range_m < 0 || range_m == INT32_MAX) return fail(FS_E_INVALID, "range out of range");
    Server &S = sv->impl;
    std::unique_ptr<Instance> I(new Instance);
    I->B = B;
    I->M = M;
    I->K = K;
    I->R = range_m;
    I->ldc = (M + 3) / 4 * 4;
    I->bases.assign(base_latlon_deg, base_latlon_deg + 2 * (size_t)B);
    I->missions.assign(mission_pd_deg, mission_pd_deg + 4 * (size_t)M);
    I->table_bytes = table_of(B, M);
    const size_t need = I->table_bytes + workspace_of(B, M, K, true);
    if ((int64_t)need > S.cfg.hbm_budget_bytes)
        return fail(FS_E_BUDGET, "instance needs %zu bytes, budget is %lld", need,
                    (long long)S.cfg.hbm_budget_bytes);
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.closing) return fail(FS_E_CLOSED, "server is closing");
    if (S.failed) return fail(FS_E_DEVICE, "server failed: %s", S.fail_msg.c_str());
    I->id = S.next_inst++;
    *instance_id = I->id;
    S.insts[I->id] = std::move(I);
    return FS_OK;
}

extern "C" fs_status fs_serve_submit(fs_server *sv, int64_t instance_id,
                                     const int32_t *mission_ids, const double *new_pd_deg,
                                     int32_t n, const fs_params *p, uint64_t *ticket)
{
    using namespace fs;
    if (!sv || !ticket) return fail(FS_E_INVALID, "NULL argument");
    if (n < 0 || (n > 0 && (!mission_ids || !new_pd_deg)))
        return fail(FS_E_INVALID, "bad mission list");
    FS_TRY(check_params(p));
    if (p->mode > 1)
        return fail(FS_E_INVALID, "the server runs modes 0 and 1 (mode %d requested)", p->mode);
    Server &S = sv->impl;
    std::unique_ptr<Request> r(new Request);
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.closing) return fail(FS_E_CLOSED, "server is closing");
    if (S.failed) return fail(FS_E_DEVICE, "server failed: %s", S.fail_msg.c_str());
    auto it = S.insts.find(instance_id);
    if (it == S.insts.end()) return fail(FS_E_NOTFOUND, "unknown instance %lld", (long long)instance_id);
    Instance &I = *it->second;
    for (int32_t q = 0; q < n; ++q)
        if (mission_ids[q] < 0 || mission_ids[q] >= I.M)
            return fail(FS_E_INVALID, "mission id %d outside [0, %d)", mission_ids[q], I.M);
    r->ticket = S.next_ticket++;
    r->inst = instance_id;
    r->I = &I;
    r->ids.assign(mission_ids, mission_ids + n);
    r->pd.assign(new_pd_deg, new_pd_deg + 4 * (size_t)n);
    r->p = *p;
    r->t_submit = Clock::now();
    *ticket = r->ticket;
    S.submitted.push_back(r.get());
    S.requests[r->ticket] = std::move(r);
    S.stats.queued += 1;
    S.cv.notify_all();
    return FS_OK;
}

extern "C" fs_status fs_serve_poll(fs_server *sv, uint64_t ticket, int32_t *open_out,
                                   fs_score *score_out, double *latency_s)
{
    using namespace fs;
    if (!sv) return fail(FS_E_INVALID, "NULL server");
    Server &S = sv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.requests.find(ticket);
    if (it == S.requests.end()) return fail(FS_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second.get();
    if (r->state != kDone) return FS_PENDING;
    const fs_status st = r->status;
    if (st == FS_OK) {
        if (open_out) std::copy(r->best.begin(), r->best.end(), open_out);
        if (score_out) *score_out = r->score;
        if (latency_s)
            *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    } else {
        fail(st, "%s", r->err.c_str());
    }
    S.requests.erase(it);
    return st;
}

extern "C" fs_status fs_serve_stats_get(fs_server *sv, fs_serve_stats *out)
{
    using namespace fs;
    if (!sv || !out) return fail(FS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->impl.mu);
    *out = sv->impl.stats;
    return FS_OK;
}

extern "C" fs_status fs_serve_close(fs_server *sv)
{
    using namespace fs;
    if (!sv) return fail(FS_E_INVALID, "NULL server");
    Server &S = sv->impl;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.closing = true;
    }
    S.cv.notify_all();
    if (S.th.joinable()) S.th.join();
    S.release_device();
    delete sv;
    return FS_OK;
}
