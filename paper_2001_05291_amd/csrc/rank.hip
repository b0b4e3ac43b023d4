// Base ranking (Section 4.1, Algorithm 1's Top_Vals).
//
// Row sums S_b = sum_m C[b][m] in int64: one workgroup per base row streams
// the row with 16-byte loads and reduces across the wavefront with DPP-backed
// shuffles (HBM-bound: B*M*4 bytes read once).  The K bases of smallest
// (S_b, b) are then selected by rank counting, which is exact and needs no
// sort network: the rank of b is the number of bases b' with
// (S_b', b') < (S_b, b).  Selection is O(B^2) compare work spread over the
// grid (16 lanes per base), a few microseconds at the few thousand bases this
// targets.
#include "fs_internal.h"

namespace fs {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(kBlock) void k_row_sums(const int32_t *__restrict__ C, int64_t ldc,
                                                     int32_t M, int vec4,
                                                     int64_t *__restrict__ sums)
{
    const int32_t b = blockIdx.x;
    const int32_t *row = C + (int64_t)b * ldc;
    int64_t acc = 0;
    if (vec4) {
        const int32_t nq = M / 4;
        const v4i *r4 = reinterpret_cast<const v4i *>(row);
        for (int32_t q = threadIdx.x; q < nq; q += kBlock) {
            const v4i v = __builtin_nontemporal_load(r4 + q);
            acc += (int64_t)v.x + v.y + (int64_t)v.z + v.w;
        }
        for (int32_t m = nq * 4 + threadIdx.x; m < M; m += kBlock) acc += row[m];
    } else {
        for (int32_t m = threadIdx.x; m < M; m += kBlock) acc += row[m];
    }
    acc = wave_sum_i64(acc);
    __shared__ int64_t part[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int w = 0; w < kBlock / 64; ++w) s += part[w];
        sums[b] = s;
    }
}

// order_out[rank(b)] = b for every b of rank < K.  A workgroup takes 16
// candidates with 16 lanes each; a lane compares its candidate with every
// 16th competitor of an LDS tile, and the 16 partial counts are summed with
// lane exchanges (250 workgroups at B = 4,000 instead of 16, each lane 250
// comparisons instead of 4,000).
constexpr int kSelLanes = 16;
constexpr int kSelTile = 2048;

__global__ __launch_bounds__(kBlock) void k_rank_select(const int64_t *__restrict__ sums, int32_t B,
                                                        int32_t K, int32_t *__restrict__ order_out)
{
    __shared__ int64_t tile[kSelTile];
    const int32_t sub = threadIdx.x % kSelLanes, cand = threadIdx.x / kSelLanes;
    const int32_t b = blockIdx.x * (kBlock / kSelLanes) + cand;
    const int64_t mine = b < B ? sums[b] : 0;
    int32_t rank = 0;
    for (int32_t t0 = 0; t0 < B; t0 += kSelTile) {
        const int32_t n = min(kSelTile, B - t0);
        __syncthreads();
        for (int32_t i = threadIdx.x; i < n; i += kBlock) tile[i] = sums[t0 + i];
        __syncthreads();
#pragma unroll 8
        for (int32_t q = sub; q < n; q += kSelLanes) {
            const int64_t o = tile[q];
            rank += (o < mine) || (o == mine && t0 + q < b);
        }
    }
#pragma unroll
    for (int off = kSelLanes / 2; off > 0; off >>= 1) rank += __shfl_xor(rank, off, 64);
    if (sub == 0 && b < B && rank < K) order_out[rank] = b;
}

// out[position of v among ids] = v: ascending order of K distinct ids.
__global__ __launch_bounds__(kBlock) void k_sort_ids(const int32_t *__restrict__ ids, int32_t K,
                                                     int32_t *__restrict__ out)
{
    const int32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= K) return;
    const int32_t v = ids[k];
    int32_t pos = 0;
    for (int32_t q = 0; q < K; ++q) pos += ids[q] < v;
    out[pos] = v;
}

}  // namespace

fs_status launch_rank(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                      int32_t *order_out, int64_t *sums, hipStream_t s)
{
    const int vec4 = (ldc % 4 == 0) && ((uintptr_t)C % 16 == 0);
    k_row_sums<<<B, kBlock, 0, s>>>(C, ldc, M, vec4, sums);
    FS_HIP(hipGetLastError());
    constexpr int per_block = kBlock / kSelLanes;
    k_rank_select<<<(B + per_block - 1) / per_block, kBlock, 0, s>>>(sums, B, K, order_out);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

fs_status launch_sort_ids(const int32_t *ids, int32_t K, int32_t *out, hipStream_t s)
{
    k_sort_ids<<<(K + kBlock - 1) / kBlock, kBlock, 0, s>>>(ids, K, out);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

}  // namespace fs

extern "C" fs_status fs_rank_bases(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                                   int32_t *open_out, int32_t *order_out, int64_t *row_sums,
                                   void *stream)
{
    using namespace fs;
    FS_TRY(check_table(C, ldc, B, M));
    if (K < 1 || K > B) return fail(FS_E_INVALID, "K=%d must be in [1, B=%d]", K, B);
    if (!open_out) return fail(FS_E_INVALID, "open_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    int64_t *sums = row_sums;
    int32_t *order = order_out;
    void *scratch = nullptr;
    size_t need = (row_sums ? 0 : sizeof(int64_t) * (size_t)B) +
                  (order_out ? 0 : sizeof(int32_t) * (size_t)K);
    if (need) {
        FS_HIP(hipMallocAsync(&scratch, need, s));
        char *p = (char *)scratch;
        if (!row_sums) {
            sums = (int64_t *)p;
            p += sizeof(int64_t) * (size_t)B;
        }
        if (!order_out) order = (int32_t *)p;
    }
    fs_status st = launch_rank(C, ldc, B, M, K, order, sums, s);
    if (st == FS_OK) st = launch_sort_ids(order, K, open_out, s);
    if (scratch) FS_HIP(hipFreeAsync(scratch, s));
    return st;
}
