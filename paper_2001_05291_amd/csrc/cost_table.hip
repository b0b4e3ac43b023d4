// Cost table: FP64 haversine round trips rounded to int32 metres.
//
// Eq. 1 (Section 3) gives the haversine great-circle distance; Section 3
// defines a mission as pickup, delivery and return to the same base, and
// Algorithm 1 (Section 4.1) fills the base-by-mission Distances table.  A
// workgroup covers 256 missions of kBasesPerBlock base rows: the per-mission
// terms (angles in radians, cosines, the pickup->delivery leg) are computed
// once by a prologue kernel, so the main kernel evaluates two haversines per
// (base, mission) entry.  The kernel is bound by FP64 VALU work (two sines,
// one square root and one arcsine per haversine), not by the int32 writes.
//
// This file is compiled with -ffp-contract=off so that every product and sum
// is rounded separately, in the order written.
#include <algorithm>

#include "fs_internal.h"

namespace fs {
namespace {

constexpr double kDeg2Rad = 3.14159265358979323846 / 180.0;
constexpr int kBasesPerBlock = 4;

struct MissionPrep {
    double *phi_p, *psi_p, *cos_p;
    double *phi_d, *psi_d, *cos_d;
    double *pd;  // pickup -> delivery leg
};

// Haversine of Eq. 1 between point a and point b, angles in radians, with the
// cosines of the latitudes precomputed.  The radicand is clamped to [0, 1].
__device__ __forceinline__ double haversine(double phi_a, double psi_a, double cos_a,
                                            double phi_b, double psi_b, double cos_b,
                                            double two_r)
{
    double s_phi = sin((phi_a - phi_b) / 2.0);
    double s_psi = sin((psi_a - psi_b) / 2.0);
    double h = s_phi * s_phi + cos_a * cos_b * (s_psi * s_psi);
    h = fmin(fmax(h, 0.0), 1.0);
    return two_r * asin(sqrt(h));
}

__global__ __launch_bounds__(kBlock) void k_mission_prep(const double *__restrict__ mpd, int32_t M,
                                                         double two_r, MissionPrep mp)
{
    int32_t m = blockIdx.x * kBlock + threadIdx.x;
    if (m >= M) return;
    const double *q = mpd + 4 * (int64_t)m;
    double phi_p = q[0] * kDeg2Rad, psi_p = q[1] * kDeg2Rad;
    double phi_d = q[2] * kDeg2Rad, psi_d = q[3] * kDeg2Rad;
    double cos_p = cos(phi_p), cos_d = cos(phi_d);
    mp.phi_p[m] = phi_p;
    mp.psi_p[m] = psi_p;
    mp.cos_p[m] = cos_p;
    mp.phi_d[m] = phi_d;
    mp.psi_d[m] = psi_d;
    mp.cos_d[m] = cos_d;
    mp.pd[m] = haversine(phi_p, psi_p, cos_p, phi_d, psi_d, cos_d, two_r);
}

// Angles and latitude cosine of the kBasesPerBlock bases from b0 on, computed
// by the block's first threads into LDS for the whole block: the values every
// thread would compute itself, at one cosine per base instead of one per
// (base, mission).  Called by every thread of the block.
__device__ __forceinline__ void stage_bases(const double *__restrict__ bases, int32_t B,
                                            int32_t b0, double (*s_base)[3])
{
    __syncthreads();   // the previous group's reads are done
    const int32_t t = threadIdx.x;
    if (t < kBasesPerBlock && b0 + t < B) {
        const double phi = bases[2 * (int64_t)(b0 + t)] * kDeg2Rad;
        s_base[t][0] = phi;
        s_base[t][1] = bases[2 * (int64_t)(b0 + t) + 1] * kDeg2Rad;
        s_base[t][2] = cos(phi);
    }
    __syncthreads();
}

// grid: x = mission blocks of kBlock, y = base groups of kBasesPerBlock.
__global__ __launch_bounds__(kBlock) void k_cost_table(const double *__restrict__ bases, int32_t B,
                                                       int32_t M, double two_r, int32_t legs,
                                                       MissionPrep mp, int32_t *__restrict__ C,
                                                       double *__restrict__ Cf, int64_t ldc)
{
    __shared__ double s_base[kBasesPerBlock][3];
    const int32_t m = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = m < M;   // no early exit: every thread takes the barriers
    double phi_p = 0, psi_p = 0, cos_p = 0, phi_d = 0, psi_d = 0, cos_d = 0, pd = 0;
    if (valid) {
        phi_p = mp.phi_p[m], psi_p = mp.psi_p[m], cos_p = mp.cos_p[m];
        phi_d = mp.phi_d[m], psi_d = mp.psi_d[m], cos_d = mp.cos_d[m];
        pd = mp.pd[m];
    }
    for (int32_t b0 = blockIdx.y * kBasesPerBlock; b0 < B; b0 += gridDim.y * kBasesPerBlock) {
        stage_bases(bases, B, b0, s_base);
        if (!valid) continue;
#pragma unroll
        for (int q = 0; q < kBasesPerBlock; ++q) {
            const int32_t b = b0 + q;
            if (b >= B) break;
            const double phi_b = s_base[q][0], psi_b = s_base[q][1], cos_b = s_base[q][2];
            const double bp = haversine(phi_b, psi_b, cos_b, phi_p, psi_p, cos_p, two_r);
            const double db = haversine(phi_d, psi_d, cos_d, phi_b, psi_b, cos_b, two_r);
            const double v = (legs == 3) ? (bp + pd) + db : bp + db;
            const int64_t at = (int64_t)b * ldc + m;
            C[at] = (int32_t)rint(v);
            if (Cf) Cf[at] = v;
        }
    }
}

// Recomputes the columns of the given missions: ids[i] receives the costs of
// the mission with coordinates mpd[i].  grid: x = id blocks, y = base groups.
// Ids outside [0, M) are skipped.
__global__ __launch_bounds__(kBlock) void k_cost_columns(const double *__restrict__ bases, int32_t B,
                                                         const int32_t *__restrict__ ids,
                                                         const double *__restrict__ mpd, int32_t n,
                                                         int32_t M, double two_r, int32_t legs,
                                                         int32_t *__restrict__ C, int64_t ldc)
{
    __shared__ double s_base[kBasesPerBlock][3];
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const int32_t m = i < n ? ids[i] : -1;
    const bool valid = m >= 0 && m < M;   // no early exit: every thread takes the barriers
    double phi_p = 0, psi_p = 0, cos_p = 0, phi_d = 0, psi_d = 0, cos_d = 0, pd = 0;
    if (valid) {
        const double *q = mpd + 4 * (int64_t)i;
        phi_p = q[0] * kDeg2Rad, psi_p = q[1] * kDeg2Rad;
        phi_d = q[2] * kDeg2Rad, psi_d = q[3] * kDeg2Rad;
        cos_p = cos(phi_p), cos_d = cos(phi_d);
        pd = haversine(phi_p, psi_p, cos_p, phi_d, psi_d, cos_d, two_r);
    }
    for (int32_t b0 = blockIdx.y * kBasesPerBlock; b0 < B; b0 += gridDim.y * kBasesPerBlock) {
        stage_bases(bases, B, b0, s_base);
        if (!valid) continue;
#pragma unroll
        for (int q2 = 0; q2 < kBasesPerBlock; ++q2) {
            const int32_t b = b0 + q2;
            if (b >= B) break;
            const double phi_b = s_base[q2][0], psi_b = s_base[q2][1], cos_b = s_base[q2][2];
            const double bp = haversine(phi_b, psi_b, cos_b, phi_p, psi_p, cos_p, two_r);
            const double db = haversine(phi_d, psi_d, cos_d, phi_b, psi_b, cos_b, two_r);
            const double v = (legs == 3) ? (bp + pd) + db : bp + db;
            C[(int64_t)b * ldc + m] = (int32_t)rint(v);
        }
    }
}

// Indexed form: missions given as (pickup, delivery) hospital ids.  Per
// mission: the pickup -> delivery leg from the hospitals' coordinates (the
// same doubles as the direct form's mission coordinates) and a check of the
// ids (bad ids are counted, and the table is not built).
constexpr int32_t kIndexedMaxH = 16384;   // one FP64 leg per hospital in LDS (128 KB)
// Workgroup size of k_cost_indexed: 768 threads while two workgroups' legs fit
// one CU's LDS (H <= 10,240), so that one workgroup's haversines overlap the
// other's stores (80 registers a thread leave room for 2 x 12 waves, not for
// 2 x 16): 0.75 -> 0.62 ms per call at 4,000 bases x 10,000 hospitals x
// 100,000 missions; 1,024 threads when one workgroup holds a CU's LDS anyway.
constexpr int kIndexedBlockPair = 768;
constexpr int kIndexedBlockOne = 1024;
constexpr size_t kLdsPerCu = 160 * 1024;

__global__ __launch_bounds__(kBlock) void k_mission_legs(const double *__restrict__ hosp,
                                                         int32_t H,
                                                         const int32_t *__restrict__ ph,
                                                         int32_t M, double two_r,
                                                         double *__restrict__ pd,
                                                         uint32_t *__restrict__ packed,
                                                         int32_t *__restrict__ bad)
{
    const int32_t m = blockIdx.x * kBlock + threadIdx.x;
    if (m >= M) return;
    const int32_t p = ph[2 * (int64_t)m], d = ph[2 * (int64_t)m + 1];
    if (p < 0 || p >= H || d < 0 || d >= H) {
        atomicAdd(bad, 1);
        pd[m] = 0.0;
        packed[m] = 0;
        return;
    }
    const double phi_p = hosp[2 * (int64_t)p] * kDeg2Rad, psi_p = hosp[2 * (int64_t)p + 1] * kDeg2Rad;
    const double phi_d = hosp[2 * (int64_t)d] * kDeg2Rad, psi_d = hosp[2 * (int64_t)d + 1] * kDeg2Rad;
    pd[m] = haversine(phi_p, psi_p, cos(phi_p), phi_d, psi_d, cos(phi_d), two_r);
    packed[m] = (uint32_t)p | ((uint32_t)d << 16);
}

// Per hospital: latitude and longitude in radians and the cosine of the
// latitude (the same expressions as in the legs above, so the same doubles).
__global__ __launch_bounds__(kBlock) void k_hosp_prep(const double *__restrict__ hosp, int32_t H,
                                                      double *__restrict__ hp)
{
    const int32_t h = blockIdx.x * kBlock + threadIdx.x;
    if (h >= H) return;
    const double phi = hosp[2 * (int64_t)h] * kDeg2Rad;
    const double psi = hosp[2 * (int64_t)h + 1] * kDeg2Rad;
    hp[h] = phi;
    hp[H + h] = psi;
    hp[2 * (int64_t)H + h] = cos(phi);
}

// One workgroup per base: the leg between the base and every hospital in LDS,
// then C[b][m] = (leg(b, p) + pd) + leg(d, b) for every mission, in the
// direct form's order.  The haversine above is symmetric bit for bit (the
// two angle differences only change sign, sin is odd, and the product of
// the cosines commutes), so one leg per hospital serves both directions and
// the table is bitwise the direct form's (tested).
template <int BS>
__global__ __launch_bounds__(BS) void k_cost_indexed(
    const double *__restrict__ bases, const double *__restrict__ hp, int32_t H,
    const double *__restrict__ pd, const uint32_t *__restrict__ packed, int32_t M, double two_r,
    int32_t legs, int32_t *__restrict__ C, double *__restrict__ Cf, int64_t ldc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *leg = reinterpret_cast<double *>(smem);   // base <-> hospital
    const int32_t b = blockIdx.x;
    const double phi_b = bases[2 * (int64_t)b] * kDeg2Rad;
    const double psi_b = bases[2 * (int64_t)b + 1] * kDeg2Rad;
    const double cos_b = cos(phi_b);
    // (hospital angles and cosines from k_hosp_prep)
    for (int32_t h = threadIdx.x; h < H; h += BS)
        leg[h] = haversine(phi_b, psi_b, cos_b, hp[h], hp[H + h], hp[2 * (int64_t)H + h], two_r);
    __syncthreads();
    const int64_t row = (int64_t)b * ldc;
    // four missions per thread and step, their loads issued together
    constexpr int U = 4;
    for (int32_t m0 = threadIdx.x; m0 < M; m0 += U * BS) {
        uint32_t q[U];
        double pdm[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t m = m0 + u * BS;
            q[u] = m < M ? packed[m] : 0u;
            pdm[u] = m < M ? pd[m] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t m = m0 + u * BS;
            if (m >= M) break;
            const double bp = leg[q[u] & 0xFFFF];
            const double db = leg[q[u] >> 16];
            const double v = (legs == 3) ? (bp + pdm[u]) + db : bp + db;
            C[row + m] = (int32_t)rint(v);
            if (Cf) Cf[row + m] = v;
        }
    }
}

}  // namespace

fs_status launch_cost_columns(const double *bases, int32_t B, const int32_t *ids,
                              const double *mpd, int32_t n, int32_t M, double radius,
                              int32_t legs, int32_t *C, int64_t ldc, hipStream_t s)
{
    if (n <= 0) return FS_OK;
    const double r = radius == 0.0 ? 6371000.0 : radius;
    const int32_t gy = std::min<int32_t>((B + kBasesPerBlock - 1) / kBasesPerBlock, 65535);
    dim3 g((n + kBlock - 1) / kBlock, gy);
    k_cost_columns<<<g, kBlock, 0, s>>>(bases, B, ids, mpd, n, M, 2.0 * r, legs, C, ldc);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

}  // namespace fs

extern "C" fs_status fs_build_cost_table(const double *base_latlon_deg, int32_t B,
                                         const double *mission_pd_deg, int32_t M,
                                         double earth_radius_m, int32_t legs, int32_t *C,
                                         int64_t ldc, double *Cf, void *stream)
{
    using namespace fs;
    if (!base_latlon_deg || !mission_pd_deg || !C)
        return fail(FS_E_INVALID, "NULL coordinate or output pointer");
    if (B < 1 || M < 1) return fail(FS_E_INVALID, "B=%d, M=%d: both must be >= 1", B, M);
    if (ldc < M) return fail(FS_E_INVALID, "row pitch ldc=%lld < M=%d", (long long)ldc, M);
    if (legs != 2 && legs != 3) return fail(FS_E_INVALID, "legs=%d: must be 2 or 3", legs);
    if (!(earth_radius_m >= 0.0)) return fail(FS_E_INVALID, "negative or NaN radius");
    double r = earth_radius_m == 0.0 ? 6371000.0 : earth_radius_m;
    if (r > 1.1e8) return fail(FS_E_INVALID, "radius %.3g m: costs would overflow int32", r);
    hipStream_t s = (hipStream_t)stream;

    MissionPrep mp{};
    double *buf = nullptr;
    FS_HIP(hipMallocAsync((void **)&buf, sizeof(double) * 7 * (size_t)M, s));
    mp.phi_p = buf;
    mp.psi_p = buf + (size_t)M;
    mp.cos_p = buf + 2 * (size_t)M;
    mp.phi_d = buf + 3 * (size_t)M;
    mp.psi_d = buf + 4 * (size_t)M;
    mp.cos_d = buf + 5 * (size_t)M;
    mp.pd = buf + 6 * (size_t)M;
    double two_r = 2.0 * r;
    dim3 g1((M + kBlock - 1) / kBlock);
    k_mission_prep<<<g1, kBlock, 0, s>>>(mission_pd_deg, M, two_r, mp);
    FS_HIP(hipGetLastError());
    int32_t gy = (B + kBasesPerBlock - 1) / kBasesPerBlock;
    dim3 g2((M + kBlock - 1) / kBlock, gy < 65535 ? gy : 65535);
    k_cost_table<<<g2, kBlock, 0, s>>>(base_latlon_deg, B, M, two_r, legs, mp, C, Cf, ldc);
    FS_HIP(hipGetLastError());
    FS_HIP(hipFreeAsync(buf, s));
    return FS_OK;
}

extern "C" fs_status fs_build_cost_table_indexed(const double *base_latlon_deg, int32_t B,
                                                 const double *hosp_latlon_deg, int32_t H,
                                                 const int32_t *mission_ph, int32_t M,
                                                 double earth_radius_m, int32_t legs, int32_t *C,
                                                 int64_t ldc, double *Cf, void *stream)
{
    using namespace fs;
    if (!base_latlon_deg || !hosp_latlon_deg || !mission_ph || !C)
        return fail(FS_E_INVALID, "NULL coordinate, id or output pointer");
    if (B < 1 || M < 1 || H < 1)
        return fail(FS_E_INVALID, "B=%d, H=%d, M=%d: all must be >= 1", B, H, M);
    if (H > kIndexedMaxH)
        return fail(FS_E_INVALID, "H=%d hospitals: the indexed form takes at most %d", H,
                    kIndexedMaxH);
    if (ldc < M) return fail(FS_E_INVALID, "row pitch ldc=%lld < M=%d", (long long)ldc, M);
    if (legs != 2 && legs != 3) return fail(FS_E_INVALID, "legs=%d: must be 2 or 3", legs);
    if (!(earth_radius_m >= 0.0)) return fail(FS_E_INVALID, "negative or NaN radius");
    const double r = earth_radius_m == 0.0 ? 6371000.0 : earth_radius_m;
    if (r > 1.1e8) return fail(FS_E_INVALID, "radius %.3g m: costs would overflow int32", r);
    hipStream_t s = (hipStream_t)stream;
    const double two_r = 2.0 * r;
    char *buf = nullptr;
    const size_t pd_bytes = sizeof(double) * (size_t)M, pk_bytes = sizeof(uint32_t) * (size_t)M;
    const size_t hp_bytes = sizeof(double) * 3 * (size_t)H;
    FS_HIP(hipMallocAsync((void **)&buf, hp_bytes + pd_bytes + pk_bytes + 256, s));
    double *hp = (double *)buf;
    double *pd = (double *)(buf + hp_bytes);
    uint32_t *packed = (uint32_t *)(buf + hp_bytes + pd_bytes);
    int32_t *bad = (int32_t *)(buf + hp_bytes + pd_bytes + pk_bytes);   // (4-aligned)
    int32_t nbad = 0;
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(int32_t), s);
    if (e == hipSuccess) {
        k_mission_legs<<<(M + kBlock - 1) / kBlock, kBlock, 0, s>>>(hosp_latlon_deg, H, mission_ph,
                                                                   M, two_r, pd, packed, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        k_hosp_prep<<<(H + kBlock - 1) / kBlock, kBlock, 0, s>>>(hosp_latlon_deg, H, hp);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && nbad == 0) {
        const size_t lds = sizeof(double) * (size_t)H;
        const bool pair = 2 * lds <= kLdsPerCu;
        const void *fn = pair ? (const void *)k_cost_indexed<kIndexedBlockPair>
                              : (const void *)k_cost_indexed<kIndexedBlockOne>;
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e == hipSuccess) {
            if (pair)
                k_cost_indexed<kIndexedBlockPair><<<B, kIndexedBlockPair, lds, s>>>(
                    base_latlon_deg, hp, H, pd, packed, M, two_r, legs, C, Cf, ldc);
            else
                k_cost_indexed<kIndexedBlockOne><<<B, kIndexedBlockOne, lds, s>>>(
                    base_latlon_deg, hp, H, pd, packed, M, two_r, legs, C, Cf, ldc);
            e = hipGetLastError();
        }
    }
    (void)hipFreeAsync(buf, s);
    if (e != hipSuccess) return fail(FS_E_DEVICE, "indexed cost table: %s", hipGetErrorString(e));
    if (nbad) return fail(FS_E_INVALID, "%d missions name a hospital outside [0, %d)", nbad, H);
    return FS_OK;
}
