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

}  // namespace fs

extern "C" const char *fs_last_error(void) { return fs::g_msg; }

extern "C" const char *fs_version(void) { return "fleetstage 0.1.0 (gfx950)"; }
