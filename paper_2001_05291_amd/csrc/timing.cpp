// Event-pair timing of the search kernel groups (diagnostics for roofline
// reporting; off by default).
#include <mutex>
#include <string>
#include <utility>

#include "fs_internal.h"

namespace fs {

namespace {
struct Group {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pairs;
};
std::mutex g_mu;
bool g_on = false;
Group g_groups[3];

int group_index(const char *name)
{
    const std::string n = name ? name : "";
    if (n == "sweep") return 0;
    if (n == "refresh") return 1;
    if (n == "finalize") return 2;
    return -1;
}

void drop_all()
{
    for (auto &g : g_groups) {
        for (auto &p : g.pairs) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
        g.pairs.clear();
    }
}
}  // namespace

bool timing_on()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_on;
}

TimedLaunch::TimedLaunch(int group, hipStream_t s) : group_(group), s_(s)
{
    if (!timing_on()) return;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) return;
    if (hipEventRecord(a_, s_) != hipSuccess) return;
    armed_ = true;
}

TimedLaunch::~TimedLaunch()
{
    if (!armed_) {
        if (a_) (void)hipEventDestroy(a_);
        if (b_) (void)hipEventDestroy(b_);
        return;
    }
    (void)hipEventRecord(b_, s_);
    std::lock_guard<std::mutex> lk(g_mu);
    g_groups[group_].pairs.emplace_back(a_, b_);
}

}  // namespace fs

extern "C" fs_status fs_timing_enable(int32_t on)
{
    using namespace fs;
    std::lock_guard<std::mutex> lk(g_mu);
    drop_all();
    g_on = on != 0;
    return FS_OK;
}

extern "C" fs_status fs_timing_read(const char *group, double *total_ms, int64_t *launches)
{
    using namespace fs;
    const int gi = group_index(group);
    if (gi < 0) return fail(FS_E_INVALID, "unknown timing group '%s'", group ? group : "(null)");
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pairs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        pairs.swap(g_groups[gi].pairs);
    }
    double sum = 0.0;
    fs_status st = FS_OK;
    for (auto &p : pairs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(p.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
        if (e != hipSuccess && st == FS_OK)
            st = fail(FS_E_DEVICE, "event timing failed: %s", hipGetErrorString(e));
        sum += ms;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (total_ms) *total_ms = sum;
    if (launches) *launches = (int64_t)pairs.size();
    return st;
}
