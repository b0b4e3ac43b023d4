// Exact optimum by enumeration: the stand-in for the exact solver column of
// the paper's evaluation (Section 5), for small instances.  Every K-subset of
// the B bases is a placement; placements are ranked in lexicographic order of
// their ascending id tuples, and the optimum is the best value under the
// placement order (coverage desc, distance asc) with the lowest rank among
// equal values.
//
// k_brute: each thread walks a block of consecutive ranks (unranked once,
// then stepped to the next combination), evaluates each placement from the
// cost table staged in LDS, and keeps its best; the workgroup reduces to one
// partial.  k_brute_final (one workgroup) reduces the partials, unranks the
// winner and writes the placement and its value.
#include <algorithm>
#include <vector>

#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kBruteBlock = 256;
constexpr int kBruteMaxK = 16;
constexpr int64_t kBruteMaxLds = 56 * 1024;   // bytes of binomials + staged table

struct BrutePart {
    int64_t dist;
    int64_t rank;   // -1: none
    int32_t cov;
    int32_t pad;
};

__device__ __forceinline__ bool brute_better(int32_t ca, int64_t da, int64_t ra, int32_t cb,
                                             int64_t db, int64_t rb)
{
    if (ra < 0) return false;
    if (rb < 0) return true;
    if (ca != cb) return ca > cb;
    if (da != db) return da < db;
    return ra < rb;
}

// binom[n * (K + 1) + k] = C(n, k) for n <= B, k <= K, one entry per thread
// by the multiplicative formula (each partial product is a binomial, so every
// division is exact).  Entries past 64 bits wrap; unranking only reads
// entries C(n, k) with n - k <= B - K, which are at most C(B, K).
__device__ void fill_binom(uint64_t *binom, int32_t B, int32_t K)
{
    for (int32_t q = threadIdx.x; q < (B + 1) * (K + 1); q += blockDim.x) {
        const int32_t n = q / (K + 1), k = q - n * (K + 1);
        uint64_t v = k <= n ? 1 : 0;
        for (int32_t i = 1; i <= k && k <= n; ++i) v = v * (uint64_t)(n - k + i) / (uint64_t)i;
        binom[q] = v;
    }
    __syncthreads();
}

// The rank-th K-subset of {0..B-1} in lexicographic order.
// rank < C(B, K) keeps x <= B - K + i, so every index stays in the table.
__device__ void unrank(int64_t rank, int32_t B, int32_t K, const uint64_t *binom, int32_t *S)
{
    uint64_t r = (uint64_t)rank;
    int32_t x = 0;
    for (int32_t i = 0; i < K; ++i) {
        // subsets whose i-th element is x, given the elements before it:
        // C(B - x - 1, K - i - 1)
        for (;;) {
            const uint64_t c = binom[(B - x - 1) * (K + 1) + (K - i - 1)];
            if (r < c) break;
            r -= c;
            ++x;
        }
        S[i] = x++;
    }
}

// Next K-subset in lexicographic order (false after the last one).
__device__ __forceinline__ bool next_subset(int32_t *S, int32_t B, int32_t K)
{
    int32_t i = K - 1;
    while (i >= 0 && S[i] == B - K + i) --i;
    if (i < 0) return false;
    ++S[i];
    for (int32_t q = i + 1; q < K; ++q) S[q] = S[q - 1] + 1;
    return true;
}

__global__ __launch_bounds__(kBruteBlock) void k_brute(const int32_t *__restrict__ C, int64_t ldc,
                                                       int32_t B, int32_t M, int32_t K,
                                                       int32_t R, int64_t total, int64_t per,
                                                       BrutePart *__restrict__ parts)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *binom = reinterpret_cast<uint64_t *>(smem);
    int32_t *tab = reinterpret_cast<int32_t *>(binom + (int64_t)(B + 1) * (K + 1));
    for (int64_t q = threadIdx.x; q < (int64_t)B * M; q += kBruteBlock) {
        const int32_t b = (int32_t)(q / M), m = (int32_t)(q - (int64_t)b * M);
        tab[q] = C[(int64_t)b * ldc + m];
    }
    fill_binom(binom, B, K);   // (its barrier also completes the table)

    int32_t best_c = 0;
    int64_t best_d = 0, best_r = -1;
    const int64_t r0 = ((int64_t)blockIdx.x * kBruteBlock + threadIdx.x) * per;
    if (r0 < total) {
        int32_t S[kBruteMaxK];
        unrank(r0, B, K, binom, S);
        const int64_t r1 = min(total, r0 + per);
        for (int64_t r = r0; r < r1; ++r) {
            int32_t cov = 0;
            int64_t dist = 0;
            for (int32_t m = 0; m < M; ++m) {
                int32_t v = INT32_MAX;
                for (int32_t k = 0; k < K; ++k) v = min(v, tab[S[k] * M + m]);
                if (v <= R) {
                    cov += 1;
                    dist += v;
                }
            }
            if (brute_better(cov, dist, r, best_c, best_d, best_r)) {
                best_c = cov;
                best_d = dist;
                best_r = r;
            }
            if (r + 1 < r1) next_subset(S, B, K);
        }
    }
    // workgroup best
    __shared__ BrutePart s_part[kBruteBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int32_t oc = __shfl_xor(best_c, off, 64);
        const int64_t od = __shfl_xor(best_d, off, 64);
        const int64_t orr = __shfl_xor(best_r, off, 64);
        if (brute_better(oc, od, orr, best_c, best_d, best_r)) {
            best_c = oc;
            best_d = od;
            best_r = orr;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_part[wave] = BrutePart{best_d, best_r, best_c, 0};
    __syncthreads();
    if (threadIdx.x == 0) {
        BrutePart b = s_part[0];
        for (int w = 1; w < kBruteBlock / 64; ++w) {
            const BrutePart &o = s_part[w];
            if (brute_better(o.cov, o.dist, o.rank, b.cov, b.dist, b.rank)) b = o;
        }
        parts[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(kBruteBlock) void k_brute_final(const BrutePart *__restrict__ parts,
                                                             int32_t nparts, int32_t B, int32_t K,
                                                             int32_t *__restrict__ best_open,
                                                             BrutePart *__restrict__ result)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *binom = reinterpret_cast<uint64_t *>(smem);
    fill_binom(binom, B, K);
    __shared__ BrutePart s_part[kBruteBlock];
    BrutePart b{0, -1, 0, 0};
    for (int32_t q = threadIdx.x; q < nparts; q += kBruteBlock) {
        const BrutePart o = parts[q];
        if (brute_better(o.cov, o.dist, o.rank, b.cov, b.dist, b.rank)) b = o;
    }
    s_part[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBruteBlock; ++w) {
            const BrutePart &o = s_part[w];
            if (brute_better(o.cov, o.dist, o.rank, b.cov, b.dist, b.rank)) b = o;
        }
        if (b.rank >= 0) {   // (every placement is evaluated, so one always is)
            int32_t S[kBruteMaxK];
            unrank(b.rank, B, K, binom, S);
            for (int32_t k = 0; k < K; ++k) best_open[k] = S[k];
        }
        *result = b;
    }
}

// C(n, k) on the host with overflow detection (false past int64).
bool host_binom(int64_t n, int64_t k, int64_t &out)
{
    if (k < 0 || k > n) {
        out = 0;
        return true;
    }
    k = std::min(k, n - k);
    __int128 v = 1;
    for (int64_t i = 1; i <= k; ++i) {
        v = v * (n - k + i) / i;
        if (v > (__int128)INT64_MAX) return false;
    }
    out = (int64_t)v;
    return true;
}

}  // namespace
}  // namespace fs

extern "C" fs_status fs_brute_optimum(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                                      int32_t K, int32_t range_m, int32_t *best_open_out,
                                      fs_score *score_out, int64_t *placements_out, void *stream)
{
    using namespace fs;
    FS_TRY(check_problem(C, ldc, B, M, K, range_m));
    if (!best_open_out || !score_out) return fail(FS_E_INVALID, "NULL output pointer");
    if (K > kBruteMaxK)
        return fail(FS_E_INVALID, "enumeration takes K <= %d (K = %d)", kBruteMaxK, K);
    const int64_t lds = 8 * (int64_t)(B + 1) * (K + 1) + 4 * (int64_t)B * M;
    if (lds > kBruteMaxLds)
        return fail(FS_E_INVALID, "enumeration stages the table in LDS: B * M = %lld too large",
                    (long long)B * M);
    int64_t total = 0;
    if (!host_binom(B, K, total) || total > ((int64_t)1 << 40))
        return fail(FS_E_INVALID, "C(%d, %d) placements is beyond enumeration", B, K);
    hipStream_t s = (hipStream_t)stream;
    // enough threads to fill the GPU, at most 64 placements per thread
    int64_t per = std::max<int64_t>(1, (total + 256 * 1024 - 1) / (256 * 1024));
    per = std::min<int64_t>(per, 64);
    int64_t threads = (total + per - 1) / per;
    const int64_t grid64 = (threads + kBruteBlock - 1) / kBruteBlock;
    if (grid64 > (1 << 24)) return fail(FS_E_INVALID, "enumeration grid too large");
    const int grid = (int)grid64;
    BrutePart *parts = nullptr, *result = nullptr;
    FS_HIP(hipMallocAsync((void **)&parts, sizeof(BrutePart) * ((size_t)grid + 1), s));
    result = parts + grid;
    k_brute<<<grid, kBruteBlock, (size_t)lds, s>>>(C, ldc, B, M, K, range_m, total, per, parts);
    hipError_t e = hipGetLastError();
    const size_t lds_final = 8 * (size_t)(B + 1) * (K + 1);
    if (e == hipSuccess)
        k_brute_final<<<1, kBruteBlock, lds_final, s>>>(parts, grid, B, K, best_open_out, result);
    if (e == hipSuccess) e = hipGetLastError();
    BrutePart host{};
    if (e == hipSuccess) e = hipMemcpyAsync(&host, result, sizeof host, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(parts, s);
    if (e != hipSuccess) return fail(FS_E_DEVICE, "enumeration: %s", hipGetErrorString(e));
    if (host.rank < 0) return fail(FS_E_INTERNAL, "enumeration found no placement");
    score_out->coverage = host.cov;
    score_out->distance = host.dist;
    score_out->best_iter = 0;
    if (placements_out) *placements_out = total;
    return FS_OK;
}
