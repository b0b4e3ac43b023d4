// fs_tabu_solve_noalloc: the single-instance solve for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid it).  Every device buffer the solve needs beyond the
// caller's inputs and outputs (instance descriptor, tile tables, open and
// closed lists with their tabu expiries, per-mission nearest / second-nearest
// state, the G / L_k accumulators, row-group candidates, search state, and the
// base ranking's row sums) is carved from one file-scope device array,
// `scratch`, of kScratchBytes.  Each GPU the library runs on holds its own
// copy until the process ends; its address on the current device is looked up
// once (hipGetSymbolAddress) and kept per device.
//
// Every call on a GPU shares that GPU's array, which keeps the last call's
// contents (the engine initialises everything it reads).  Calls that overlap
// on one GPU race: callers serialise them.
#include <mutex>

#include "launchset.h"

namespace fs {
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use,
// with the device current).
fs_status scratch_on_current_device(void **out)
{
    int dev = -1;
    FS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(FS_E_DEVICE, "device %d outside the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        FS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || (uintptr_t)p % 256 != 0)
            return fail(FS_E_DEVICE, "scratch array address %p is not 256-byte aligned", p);
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return FS_OK;
}

// Timing stays off for the calling thread during a call (timed launches
// would create events).
struct NoTiming {
    NoTiming() { timing_suppress(true); }
    ~NoTiming() { timing_suppress(false); }
};

}  // namespace
}  // namespace fs

extern "C" int64_t fs_noalloc_scratch_bytes(void) { return (int64_t)fs::kScratchBytes; }

extern "C" fs_status fs_tabu_solve_noalloc(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                                           int32_t K, const fs_params *p,
                                           const int32_t *init_open, int32_t *best_open_out,
                                           fs_score *score_out, int32_t *assign_out,
                                           fs_trace_rec *trace_out, void *stream)
{
    using namespace fs;
    void *base = nullptr;
    FS_TRY(scratch_on_current_device(&base));
    Workspace ws;
    ws.p = base;
    ws.cap = kScratchBytes;
    NoTiming quiet;
    return tabu_solve_impl(C, ldc, B, M, K, p, init_open, best_open_out, score_out, assign_out,
                           trace_out, (hipStream_t)stream, &ws);
}
