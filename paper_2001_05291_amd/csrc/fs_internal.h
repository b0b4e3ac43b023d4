// Internal declarations shared by the translation units of libfleetstage.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <vector>

#include "fleetstage.h"

namespace fs {

// ---------------------------------------------------------------- errors

void set_error(const char *fmt, ...);
fs_status fail(fs_status code, const char *fmt, ...);

#define FS_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t fs_e_ = (call);                                                     \
        if (fs_e_ != hipSuccess)                                                       \
            return ::fs::fail(FS_E_DEVICE, "%s failed: %s (%s:%d)", #call,             \
                              hipGetErrorString(fs_e_), __FILE__, __LINE__);           \
    } while (0)

#define FS_TRY(expr)                                                                   \
    do {                                                                               \
        fs_status fs_s_ = (expr);                                                      \
        if (fs_s_ != FS_OK) return fs_s_;                                              \
    } while (0)

// ---------------------------------------------------------------- timing

// RAII bracket of one launch of a kernel group (0 sweep, 1 refresh,
// 2 finalize) with HIP events when timing is enabled; a no-op otherwise.
bool timing_on();
// Timing of the calling thread's launches is skipped while suppressed.
void timing_suppress(bool on);
// While set (non-null), the calling thread's next timed launch stamps this
// caller-owned event pair instead of recording into a group (the autotuner's
// trial launches).
void timing_borrow(hipEvent_t start, hipEvent_t stop);

class TimedLaunch {
  public:
    // Events for one launch (or a chain of launches) of a group when timing
    // is on, else null events.  They go to hipExtLaunchKernelGGL, which has
    // the dispatch itself stamp its start and end, so timing adds no packet
    // between kernels.  Call used() once they have been handed to a launch.
    explicit TimedLaunch(int group);
    ~TimedLaunch();
    TimedLaunch(const TimedLaunch &) = delete;
    TimedLaunch &operator=(const TimedLaunch &) = delete;
    hipEvent_t start() const { return a_; }
    hipEvent_t stop() const { return b_; }
    void used() { used_ = a_ != nullptr; }

  private:
    int group_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    bool used_ = false;
    bool borrowed_ = false;
};

// ---------------------------------------------------------------- limits

constexpr int kMaxK = 1024;          // open slots handled by the sweep's LDS bins
constexpr int kBlock = 256;          // threads per workgroup of the streaming kernels
constexpr int kWideBlock = 1024;     // sweep workgroups when there are few row groups

// ---------------------------------------------------------------- device state

// Score of a placement: (coverage, distance of covered missions).
struct Score {
    int32_t cov;
    int32_t pad;
    int64_t dist;
};

// Best admissible move found by one sweep workgroup (or none: valid == 0).
struct Candidate {
    int32_t cov;             // covered missions of the moved placement; -1: no move
    int32_t i_base, j_base;  // move: base i leaves, base j enters
    uint32_t slots;          // position of i in the open list (low kSlotBits bits) and
                             // of j in the closed list (the rest)
    int64_t dist;
    uint64_t key;            // permuted searches: the move's priority in the pass (else 0)
};
static_assert(sizeof(Candidate) == 32, "candidate layout");
constexpr int kSlotBits = 10;                       // open slots: K <= kMaxK = 1 << 10
constexpr int32_t kMaxClosed = 1 << (32 - kSlotBits);   // closed slots per instance

// Per-solve search state, resident in device memory.
struct SolveState {
    int32_t stopped;    // local search reached a local optimum
    int32_t pass;       // permuted searches: the pass (scan order) in progress
    int32_t cur_cov;
    int32_t best_cov;
    int64_t cur_dist;
    int64_t best_dist;
    int32_t best_iter;
    int32_t error;      // refreshed value disagreed with the executed move's score
    int32_t err_iter;
    int32_t have_last;  // permuted searches: this pass has accepted a move ...
    uint64_t last_key;  // ... whose priority was last_key
    int32_t score_done; // fused score + refresh launches: block-scoring workgroups
                        // finished so far (each adds 1 after its candidate)
    int32_t pad;
};

// Accumulator of the per-placement sums: slot 0 is G (the placement's value),
// slot 1 + k is L_k (value change if open slot k's base is removed and its
// missions fall back to their second-nearest open base).  Two's complement in
// unsigned 64-bit so that integer atomics add signed deltas exactly.
// Each slot fills a 128-byte line of its own: the refresh workgroups add
// into these with device-scope atomics, and atomics into slots that shared a
// line were served one after another (padding took 4 us off each refresh at
// 100,000 missions and 64 vehicles).
struct Acc {
    unsigned long long cov;
    unsigned long long dist;
    unsigned long long pad[14];
};

// Host-side validation helpers.
fs_status check_table(const int32_t *C, int64_t ldc, int32_t B, int32_t M);
fs_status check_open_list(const std::vector<int32_t> &ids, int32_t B);
fs_status check_problem(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K, int32_t R);
fs_status check_params(const fs_params *p);
// Device-resident list of K ids -> host (synchronises the stream), validated.
fs_status fetch_open_list(const int32_t *dev, int32_t K, int32_t B, std::vector<int32_t> &out,
                          hipStream_t s);
// Prefixes the current message with "<what> <index>: " and returns code.
fs_status prefix_error(fs_status code, const char *what, int32_t index);

// Base ranking on the device (rank.hip): row sums, then the K smallest
// (sum, id) in rank order.
fs_status launch_sort_ids(const int32_t *ids, int32_t K, int32_t *out, hipStream_t s);
fs_status launch_rank(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                      int32_t *order_out, int64_t *sums, hipStream_t s);

// Cost-table columns of changed missions (cost_table.hip): column ids[i]
// gets the round-trip costs of the mission with coordinates mpd[i] (device
// arrays); ids outside [0, M) are skipped.
fs_status launch_cost_columns(const double *bases, int32_t B, const int32_t *ids,
                              const double *mpd, int32_t n, int32_t M, double radius,
                              int32_t legs, int32_t *C, int64_t ldc, hipStream_t s);

}  // namespace fs
