// Event-pair timing of the search kernel groups (diagnostics for roofline
// reporting; off by default).  The events are stamped by the kernel dispatches
// themselves (hipExtLaunchKernel), so enabling timing does not insert marker
// packets between the kernels it measures (the runtime still spaces out a
// dispatch that carries events, so callers may time only every n-th launch).
// Events come from a pool and are
// recycled as soon as their launch has finished, so a timed loop of many
// thousand launches neither creates events nor holds them all.
#include <deque>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fs_internal.h"

namespace fs {

namespace {
struct Group {
    std::deque<std::pair<hipEvent_t, hipEvent_t>> pending;   // not yet read back
    double total_ms = 0.0;
    int64_t launches = 0;
    fs_status error = FS_OK;
};
std::mutex g_mu;
int32_t g_period = 0;          // 0: off; n: time every n-th launch of each group
int64_t g_count[4] = {0, 0, 0, 0};
Group g_groups[4];
std::vector<hipEvent_t> g_free;

constexpr size_t kKeepPending = 64;   // read back older pairs beyond this many

int group_index(const char *name)
{
    const std::string n = name ? name : "";
    if (n == "sweep") return 0;
    if (n == "refresh") return 1;
    if (n == "finalize") return 2;
    if (n == "score_refresh") return 3;
    return -1;
}

// Under g_mu.  Adds the pair's time to the group and recycles its events;
// false when its end has not been reached yet (and wait is false).
bool settle(Group &g, std::pair<hipEvent_t, hipEvent_t> p, bool wait)
{
    hipError_t e = wait ? hipEventSynchronize(p.second) : hipEventQuery(p.second);
    if (e == hipErrorNotReady) return false;
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
    if (e != hipSuccess && g.error == FS_OK)
        g.error = fail(FS_E_DEVICE, "event timing failed: %s", hipGetErrorString(e));
    g.total_ms += ms;
    g.launches += 1;
    g_free.push_back(p.first);
    g_free.push_back(p.second);
    return true;
}

void reset_all()
{
    for (auto &g : g_groups) {
        for (auto &p : g.pending) {
            (void)hipEventSynchronize(p.second);
            g_free.push_back(p.first);
            g_free.push_back(p.second);
        }
        g.pending.clear();
        g.total_ms = 0.0;
        g.launches = 0;
        g.error = FS_OK;
    }
    for (auto &c : g_count) c = 0;
}

hipEvent_t take_event()
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_free.empty()) {
            hipEvent_t e = g_free.back();
            g_free.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void give_event(hipEvent_t e)
{
    if (!e) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_free.push_back(e);
}
}  // namespace

thread_local bool t_suppressed = false;
thread_local hipEvent_t t_borrow_a = nullptr, t_borrow_b = nullptr;

void timing_suppress(bool on) { t_suppressed = on; }

void timing_borrow(hipEvent_t start, hipEvent_t stop)
{
    t_borrow_a = start;
    t_borrow_b = stop;
}

bool timing_on()
{
    if (t_suppressed) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_period > 0;
}

namespace {
// Whether this launch of the group is one of the sampled ones.
bool sample_launch(int group)
{
    if (t_suppressed) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_period <= 0) return false;
    return g_count[group]++ % g_period == 0;
}
}  // namespace

TimedLaunch::TimedLaunch(int group) : group_(group)
{
    if (t_borrow_a) {
        a_ = t_borrow_a;
        b_ = t_borrow_b;
        borrowed_ = true;
        return;
    }
    if (!sample_launch(group)) return;
    a_ = take_event();
    b_ = take_event();
    if (!a_ || !b_) {
        give_event(a_);
        give_event(b_);
        a_ = b_ = nullptr;
    }
}

TimedLaunch::~TimedLaunch()
{
    if (borrowed_) return;
    if (!used_) {
        give_event(a_);
        give_event(b_);
        return;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    Group &g = g_groups[group_];
    g.pending.emplace_back(a_, b_);
    while (g.pending.size() > kKeepPending && settle(g, g.pending.front(), false))
        g.pending.pop_front();
}

}  // namespace fs

extern "C" fs_status fs_timing_enable(int32_t on)
{
    using namespace fs;
    std::lock_guard<std::mutex> lk(g_mu);
    if (on < 0) return fail(FS_E_INVALID, "timing period %d is negative", on);
    reset_all();
    g_period = on;
    return FS_OK;
}

extern "C" fs_status fs_timing_read(const char *group, double *total_ms, int64_t *launches)
{
    using namespace fs;
    const int gi = group_index(group);
    if (gi < 0) return fail(FS_E_INVALID, "unknown timing group '%s'", group ? group : "(null)");
    std::lock_guard<std::mutex> lk(g_mu);
    Group &g = g_groups[gi];
    while (!g.pending.empty()) {
        settle(g, g.pending.front(), true);
        g.pending.pop_front();
    }
    if (total_ms) *total_ms = g.total_ms;
    if (launches) *launches = g.launches;
    const fs_status st = g.error;
    g.total_ms = 0.0;
    g.launches = 0;
    g.error = FS_OK;
    return st;
}
