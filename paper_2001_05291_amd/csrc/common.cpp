// Error reporting, version and host-side validation shared by the entry points.
#include <cstdio>
#include <cstring>

#include "fs_internal.h"

namespace fs {

namespace {
thread_local char g_msg[512] = "";
}

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
}

fs_status fail(fs_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
    return code;
}

fs_status check_table(const int32_t *C, int64_t ldc, int32_t B, int32_t M)
{
    if (!C) return fail(FS_E_INVALID, "cost table pointer is NULL");
    if (B < 1) return fail(FS_E_INVALID, "B=%d: need at least one base", B);
    if (M < 1) return fail(FS_E_INVALID, "M=%d: need at least one mission", M);
    if (ldc < M) return fail(FS_E_INVALID, "row pitch ldc=%lld is smaller than M=%d",
                             (long long)ldc, M);
    if (ldc > (int64_t)1 << 40) return fail(FS_E_INVALID, "row pitch ldc=%lld too large",
                                            (long long)ldc);
    return FS_OK;
}

fs_status check_open_list(const std::vector<int32_t> &ids, int32_t B)
{
    std::vector<unsigned char> seen((size_t)B, 0);
    for (size_t k = 0; k < ids.size(); ++k) {
        int32_t b = ids[k];
        if (b < 0 || b >= B)
            return fail(FS_E_INVALID, "open base id %d at slot %zu is outside [0, %d)", b, k, B);
        if (seen[(size_t)b]) return fail(FS_E_INVALID, "open base id %d appears twice", b);
        seen[(size_t)b] = 1;
    }
    return FS_OK;
}

fs_status check_problem(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K, int32_t R)
{
    FS_TRY(check_table(C, ldc, B, M));
    if (K < 1 || K > B) return fail(FS_E_INVALID, "K=%d must be in [1, B=%d]", K, B);
    if (K > kMaxK) return fail(FS_E_INVALID, "K=%d exceeds the supported %d vehicles", K, kMaxK);
    if (B - K >= kMaxClosed)
        return fail(FS_E_INVALID, "B - K = %d closed bases exceed the supported %d", B - K,
                    kMaxClosed - 1);
    if (R < 0 || R == INT32_MAX) return fail(FS_E_INVALID, "range %d outside [0, INT32_MAX)", R);
    if ((int64_t)M + 3 > INT32_MAX) return fail(FS_E_INVALID, "M=%d too large", M);
    return FS_OK;
}

fs_status check_params(const fs_params *p)
{
    if (!p) return fail(FS_E_INVALID, "params pointer is NULL");
    if (p->tenure < 0) return fail(FS_E_INVALID, "tenure %d < 0", p->tenure);
    if (p->iterations < 0) return fail(FS_E_INVALID, "iterations %d < 0", p->iterations);
    if ((int64_t)p->iterations + p->tenure >= INT32_MAX)
        return fail(FS_E_INVALID, "iterations + tenure overflow int32");
    if (p->mode < 0 || p->mode > 3) return fail(FS_E_INVALID, "mode %d not in 0..3", p->mode);
    return FS_OK;
}

fs_status fetch_open_list(const int32_t *dev, int32_t K, int32_t B, std::vector<int32_t> &out,
                          hipStream_t s)
{
    out.assign(K, 0);
    FS_HIP(hipMemcpyAsync(out.data(), dev, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    return check_open_list(out, B);
}

fs_status prefix_error(fs_status code, const char *what, int32_t index)
{
    char copy[sizeof g_msg];
    snprintf(copy, sizeof copy, "%s", g_msg);
    return fail(code, "%s %d: %s", what, index, copy);
}

}  // namespace fs

extern "C" const char *fs_last_error(void) { return fs::g_msg; }

extern "C" const char *fs_version(void) { return "fleetstage 0.1.0 (gfx950)"; }
