// Tabu search over swap moves on gfx950 (Section 4.3, Algorithm 3; local-search
// baseline of Section 4.2, Algorithm 2) for any set of instances.
//
// Every check of Algorithms 2-3 recomputes the total distance of a changed
// placement, O(M) per move.  Here one iteration scores all K*(B-K) swaps
// exactly with one streaming pass over the closed rows of the cost table:
//
//   per mission m:  b1 = nearest open cost, o1 = its slot, b2 = second-nearest
//   G   = sum_m g(b1)                        (value of the placement)
//   L_i = sum_{o1(m)=i} g(b2) - g(b1)        (value change if i is closed)
//   score(i, j) = G + L_i + sum_m [g(min(c, b1)) - g(b1)]
//                         + sum_{o1(m)=i, c < b2} [g(max(c, b1)) - g(b2)]
//   with c = C[j][m] and g(v) = (v <= R) ? (1, v) : (0, 0)
//
// which equals the value of S - i + j.  Both sums vanish unless c < b2, so a
// row element costs a load and a compare on the common path; the rare path
// adds the first sum to per-lane registers and the second to an LDS bin of
// the out-slot o1(m).  One read of row j thus serves all K out-bases.
//
// One iteration is two kernels over tile tables that span every instance of
// the launch set, with no device-wide synchronisation inside either:
//   k_sweep    J closed rows x one mission chunk per workgroup; unsplit
//              instances also score their J*K moves and store the row group's
//              best admissible move (split instances go through k_score);
//   k_refresh  every workgroup reduces the instance's row-group candidates to
//              the chosen move (a few KB from L2, recomputed redundantly so no
//              workgroup waits for another), applies it to its own copy of the
//              open list and computes the nearest / second-nearest open cost
//              of its 64 missions and their share of G and L_k; the
//              workgroup of mission tile 0 also commits the move: lists for
//              the next iteration, tabu list, best-so-far and trace.
#include <algorithm>
#include <cstdlib>

#include <hip/hip_ext.h>

#include "engine.h"

namespace fs {

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    return atoi(v);
}

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned long long u64;
// Global-memory views of device pointers: loads through them are global
// loads, counted by vmcnt alone, so waiting for an LDS result does not also
// wait for them (generic loads count against both counters).
typedef const __attribute__((address_space(1))) int32_t gi32;
typedef const __attribute__((address_space(1))) v4i gv4i;
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}
// Whole-struct load / store through a global view, one dword at a time
// (merged into wide accesses by the compiler).
template <typename T>
__device__ __forceinline__ T gload(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "dword-sized structs only");
    T out;
    const gi32 *q = (const gi32 *)p;
    int32_t *o = reinterpret_cast<int32_t *>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = q[i];
    return out;
}
template <typename T>
__device__ __forceinline__ void gstore(T *p, const T &v)
{
    static_assert(sizeof(T) % 4 == 0, "dword-sized structs only");
    __attribute__((address_space(1))) int32_t *q = gptr(reinterpret_cast<int32_t *>(p));
    const int32_t *w = reinterpret_cast<const int32_t *>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) q[i] = w[i];
}

// Relaxed device-scope atomic add through a global view (no returned value).
template <typename T>
__device__ __forceinline__ void gatomic_add(T *p, T v)
{
    (void)__hip_atomic_fetch_add(gptr(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ bool better(int32_t ca, int64_t da, int32_t cb, int64_t db)
{
    return ca != cb ? ca > cb : da < db;
}

// Move order: coverage desc, distance asc, out-base asc, in-base asc.
// The move order: permuted searches (KEYED) take the lowest priority (keys
// are distinct within a pass); the other modes take coverage desc, distance
// asc, out-base asc, in-base asc (their keys are all 0).
__device__ __forceinline__ Candidate no_cand()
{
    Candidate c;
    c.cov = -1;
    c.i_base = c.j_base = 0;
    c.slots = 0;
    c.dist = 0;
    c.key = 0;
    return c;
}
__device__ __forceinline__ bool cand_valid(const Candidate &c) { return c.cov >= 0; }
__device__ __forceinline__ int32_t cand_i_slot(const Candidate &c)
{
    return (int32_t)(c.slots & ((1u << kSlotBits) - 1));
}
__device__ __forceinline__ int32_t cand_j_slot(const Candidate &c)
{
    return (int32_t)(c.slots >> kSlotBits);
}

template <bool KEYED>
__device__ __forceinline__ bool cand_better(const Candidate &a, const Candidate &b)
{
    if (!cand_valid(a)) return false;
    if (!cand_valid(b)) return true;
    if (KEYED) return a.key < b.key;
    if (a.cov != b.cov) return a.cov > b.cov;
    if (a.dist != b.dist) return a.dist < b.dist;
    if (a.i_base != b.i_base) return a.i_base < b.i_base;
    return a.j_base < b.j_base;
}

__device__ __forceinline__ int32_t wave_sum_i32(int32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <bool KEYED>
__device__ __forceinline__ Candidate shfl_xor_cand(const Candidate &c, int off)
{
    Candidate o;
    o.cov = __shfl_xor(c.cov, off, 64);
    o.i_base = __shfl_xor(c.i_base, off, 64);
    o.j_base = __shfl_xor(c.j_base, off, 64);
    o.slots = (uint32_t)__shfl_xor((int32_t)c.slots, off, 64);
    o.dist = __shfl_xor(c.dist, off, 64);
    o.key = KEYED ? __shfl_xor(c.key, off, 64) : c.key;
    return o;
}

// Best candidate of the wave under the move order (a total order, so the
// result does not depend on the reduction order); the same in every lane.
template <bool KEYED>
__device__ __forceinline__ Candidate wave_best(Candidate c)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const Candidate o = shfl_xor_cand<KEYED>(c, off);
        if (cand_better<KEYED>(o, c)) c = o;
    }
    return c;
}

// Scan orders of the permuted searches: the SplitMix64 output function
// (Steele, Lea and Flood, OOPSLA 2014) over counters.  The priority of swap
// (i out, j in) in pass p is mix64(z_p + (i B + j + 1) G) with
// z_p = mix64(seed + (p + 1) G); for fixed z_p it is injective in (i, j).
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The workgroup's tile: from the table, or (tiles == NULL: one instance,
// tiles row group major and mission chunk minor) from the block index, so
// that the descriptor load does not wait for a tile load.
__device__ __forceinline__ Tile sweep_tile(const InstDesc *descs, const Tile *tiles)
{
    if (tiles) return tiles[blockIdx.x];
    const int32_t ns = descs[0].nsplit;
    const int32_t g = (int32_t)blockIdx.x / ns;
    return Tile{0, g, (int32_t)blockIdx.x - g * ns, 0};
}

__device__ __forceinline__ Tile group_tile(const Tile *tiles)
{
    if (tiles) return tiles[blockIdx.x];
    return Tile{0, (int32_t)blockIdx.x, 0, 0};
}

// Best candidate of the workgroup under the move order (a total order, so the
// result does not depend on the reduction order); valid in every thread.
template <int BS, bool KEYED>
__device__ Candidate block_best(Candidate c, Candidate *s_red /* BS/64 + 1 */)
{
    c = wave_best<KEYED>(c);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_red[wave] = c;
    __syncthreads();
    // the waves' bests reduced across the lanes of the first wave (kept in
    // registers: a loop over s_red in one thread spills the candidate)
    constexpr int NW = BS / 64;
    static_assert((NW & (NW - 1)) == 0, "block size: a power-of-two number of waves");
    if (wave == 0) {
        Candidate b = lane < NW ? s_red[lane] : no_cand();
#pragma unroll
        for (int off = NW / 2; off > 0; off >>= 1) {
            const Candidate o = shfl_xor_cand<KEYED>(b, off);
            if (cand_better<KEYED>(o, b)) b = o;
        }
        if (lane == 0) s_red[NW] = b;
    }
    __syncthreads();
    return s_red[NW];
}

// G (k = 0) or L_{k-1}: sum of the accumulator stripes.
__device__ __forceinline__ void acc_sum(const Acc *acc, int32_t K, int32_t k, int32_t &c,
                                        int64_t &dd)
{
    u64 sc = 0, sd = 0;
    const Acc *ga = acc;
#pragma unroll
    for (int s = 0; s < kStripes; ++s) {
        sc += ga[s * (K + 1) + k].cov;
        sd += ga[s * (K + 1) + k].dist;
    }
    c = (int32_t)(int64_t)sc;
    dd = (int64_t)sd;
}

// ---------------------------------------------------------------- setup

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kBlock)
        p[q] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill_i64(int64_t *p, int64_t n, int64_t v)
{
    for (int64_t q = blockIdx.x * (int64_t)kBlock + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kBlock)
        p[q] = v;
}

// grid = ninst x per_inst blocks: tabu list, both accumulators, state.
__global__ __launch_bounds__(kBlock) void k_reset(const InstDesc *__restrict__ descs, int per_inst)
{
    const int inst = blockIdx.x / per_inst, blk = blockIdx.x - inst * per_inst;
    const InstDesc &d = descs[inst];
    if (!d.active) return;
    const int32_t q = blk * kBlock + threadIdx.x;
    if (q < d.K) {
        d.open_tabu[q] = 0;
        d.open_rot[q] = 1;   // homogeneous fleets: every vehicle rotary-wing on an
        d.open_hel[q] = 0;   // aerodrome (the typed list kernels overwrite these)
    }
    if (q < max(d.nclosed, 1)) {
        d.closed_tabu[q] = 0;
        d.closed_hel[q] = 0;
    }
    if (q < kStripes * (d.K + 1)) {
        d.acc[0][q].cov = 0;
        d.acc[0][q].dist = 0;
        d.acc[1][q].cov = 0;
        d.acc[1][q].dist = 0;
    }
    if (q == 0) *d.st = SolveState{};
}

// ---------------------------------------------------------------- ranking (A1)

// Row sums of (instance, row) tiles with 4-byte loads (rows of any pitch).
__global__ __launch_bounds__(kBlock) void k_rank_rows(const InstDesc *__restrict__ descs,
                                                      const Tile *__restrict__ tiles)
{
    const Tile tl = tiles[blockIdx.x];
    const InstDesc &d = descs[tl.inst];
    if (!d.active || !d.need_rank) return;
    const int32_t *row = d.C + (int64_t)tl.g * d.ldc;
    int64_t acc = 0;
    for (int32_t m = threadIdx.x; m < d.M; m += kBlock) acc += row[m];
    acc = wave_sum_i64(acc);
    __shared__ int64_t part[kBlock / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t sum = 0;
        for (int w = 0; w < kBlock / 64; ++w) sum += part[w];
        d.sums[tl.g] = sum;
    }
}

// One workgroup per instance: rank of every base by (sum, id); the K of rank
// < K form the open list of S_1, the others its closed list, both in
// ascending id order (the lists the single-instance path builds on the host).
// Sums are compared from LDS tiles; positions come from a prefix count.
// Exclusive prefix of one count per thread (thread 0 runs the 256-entry scan);
// returns this thread's offset and sets *total.  Every thread must call it.
__device__ int32_t block_exclusive(int32_t v, int32_t *s_cnt, int32_t *total)
{
    __syncthreads();
    s_cnt[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int w = 0; w < kBlock; ++w) {
            const int32_t c = s_cnt[w];
            s_cnt[w] = run;
            run += c;
        }
        s_cnt[kBlock] = run;
    }
    __syncthreads();
    const int32_t r = s_cnt[threadIdx.x];
    *total = s_cnt[kBlock];
    return r;
}

// Typed base ranking (heterogeneous fleet, Algorithm 1's helipad quota): walking
// the bases in (row sum, id) order, a heliport is taken only while fewer than
// K_r heliports are; the first K bases so taken are chosen.  Slots: the chosen
// heliports first, then the chosen aerodromes, each in rank order; vehicles:
// rotary-wing on the heliports and on the first K_r - (heliports chosen)
// aerodromes, fixed-wing on the rest.  Each thread walks a contiguous run of
// rank positions; the running counts come from block prefixes.  Sets sel[b].
__device__ void rank_typed(const InstDesc &d, unsigned char *sel, int32_t *s_cnt)
{
    const int32_t B = d.B, K = d.K, Kr = d.K_r;
    const int32_t *ord = d.rank_order;
    const int32_t *hel = d.base_hel;
    const int32_t per = (B + kBlock - 1) / kBlock;
    const int32_t lo = min(B, (int32_t)threadIdx.x * per), hi = min(B, lo + per);
    int32_t tot;
    // heliports before each rank position
    int32_t nh = 0;
    for (int32_t r = lo; r < hi; ++r) nh += hel[ord[r]] != 0;
    const int32_t h0 = block_exclusive(nh, s_cnt, &tot);
    // eligible bases (aerodromes, and the first K_r heliports) before each position
    int32_t ne = 0, h = h0;
    for (int32_t r = lo; r < hi; ++r) {
        const int32_t hb = hel[ord[r]] != 0;
        ne += !hb || h < Kr;
        h += hb;
    }
    const int32_t e0 = block_exclusive(ne, s_cnt, &tot);
    // chosen heliports / aerodromes before each position
    int32_t ch = 0, ca = 0;
    h = h0;
    int32_t e = e0;
    for (int32_t r = lo; r < hi; ++r) {
        const int32_t hb = hel[ord[r]] != 0;
        const bool elig = !hb || h < Kr;
        if (elig && e < K) {
            ch += hb;
            ca += !hb;
        }
        e += elig;
        h += hb;
    }
    int32_t n_hel;
    const int32_t ch0 = block_exclusive(ch, s_cnt, &n_hel);
    const int32_t ca0 = block_exclusive(ca, s_cnt, &tot);
    h = h0;
    e = e0;
    ch = ch0;
    ca = ca0;
    const int32_t rot_aero = Kr - n_hel;
    for (int32_t r = lo; r < hi; ++r) {
        const int32_t b = ord[r];
        const int32_t hb = hel[b] != 0;
        const bool elig = !hb || h < Kr;
        if (elig && e < K) {
            int32_t slot, rot;
            if (hb) {
                slot = ch++;
                rot = 1;
            } else {
                slot = n_hel + ca;
                rot = ca < rot_aero;
                ++ca;
            }
            d.open[slot] = b;
            d.open_rot[slot] = rot;
            sel[b] = 1;
        }
        e += elig;
        h += hb;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_rank_lists(const InstDesc *__restrict__ descs)
{
    const InstDesc &d = descs[blockIdx.x];
    if (!d.active || !d.need_rank) return;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *sel = smem;   // B flags
    __shared__ int64_t tile[kBlock];
    __shared__ int32_t s_cnt[kBlock + 1];
    const int32_t B = d.B, K = d.K;
    for (int32_t b0 = 0; b0 < B; b0 += kBlock) {
        const int32_t b = b0 + threadIdx.x;
        const int64_t mine = b < B ? d.sums[b] : 0;
        int32_t rank = 0;
        for (int32_t t0 = 0; t0 < B; t0 += kBlock) {
            __syncthreads();
            if (t0 + (int32_t)threadIdx.x < B) tile[threadIdx.x] = d.sums[t0 + threadIdx.x];
            __syncthreads();
            const int32_t n = min(kBlock, B - t0);
            for (int32_t q = 0; q < n; ++q) {
                const int64_t o = tile[q];
                rank += (o < mine) || (o == mine && t0 + q < b);
            }
        }
        if (b < B) {
            sel[b] = !d.typed && rank < K;
            if (d.typed) d.rank_order[rank] = b;
        }
    }
    __syncthreads();
    if (d.typed) rank_typed(d, sel, s_cnt);
    const int32_t per = (B + kBlock - 1) / kBlock;
    const int32_t lo = min(B, (int32_t)threadIdx.x * per), hi = min(B, lo + per);
    int32_t cnt = 0;
    for (int32_t b = lo; b < hi; ++b) cnt += sel[b];
    s_cnt[threadIdx.x] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int w = 0; w < kBlock; ++w) {
            const int32_t c = s_cnt[w];
            s_cnt[w] = run;
            run += c;
        }
    }
    __syncthreads();
    int32_t before = s_cnt[threadIdx.x];
    int32_t *op = d.open, *cl = d.closed;
    for (int32_t b = lo; b < hi; ++b) {
        if (sel[b]) {
            if (!d.typed) op[before] = b;   // typed: slot order set by rank_typed
            ++before;
        } else {
            cl[b - before] = b;
        }
    }
}

// Heterogeneous fleets: heliport flags beside both lists, and the vehicle types
// of a given initial placement.  grid = ninst; after the lists are in place.
__global__ __launch_bounds__(kBlock) void k_fleet_lists(const InstDesc *__restrict__ descs)
{
    const InstDesc &d = descs[blockIdx.x];
    if (!d.active || !d.typed) return;
    for (int32_t k = threadIdx.x; k < d.K; k += kBlock) {
        d.open_hel[k] = d.base_hel[d.open[k]] != 0;
        if (d.init_rot) d.open_rot[k] = d.init_rot[k] != 0;
    }
    for (int32_t q = threadIdx.x; q < d.nclosed; q += kBlock)
        d.closed_hel[q] = d.base_hel[d.closed[q]] != 0;
}

// The value of lane (lane ^ J) of a full wave.  J = 1, 2 and 8 stay in the
// vector ALU (DPP quad permutes and a rotate by 8 within each 16-lane row);
// the other distances go through the LDS crossbar.  Every lane must be
// active.
template <int J>
__device__ __forceinline__ uint64_t lane_xor64(uint64_t v)
{
    if constexpr (J == 1 || J == 2 || J == 8) {
        constexpr int kCtrl = J == 1 ? 0xB1 : (J == 2 ? 0x4E : 0x128);
        const int32_t lo = __builtin_amdgcn_update_dpp(0, (int32_t)v, kCtrl, 0xF, 0xF, false);
        const int32_t hi =
            __builtin_amdgcn_update_dpp(0, (int32_t)(v >> 32), kCtrl, 0xF, 0xF, false);
        return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    } else {
        return __shfl_xor(v, J, 64);
    }
}

template <int J>
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v)
{
    if constexpr (J == 1 || J == 2 || J == 8) {
        constexpr int kCtrl = J == 1 ? 0xB1 : (J == 2 ? 0x4E : 0x128);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, kCtrl, 0xF, 0xF, false);
    } else {
        return (uint32_t)__shfl_xor((int32_t)v, J, 64);
    }
}

__device__ __forceinline__ uint32_t lane_xor32(uint32_t v, int j)
{
    switch (j) {   // (j is a constant once the sorting network is unrolled)
    case 1: return lane_xor32<1>(v);
    case 2: return lane_xor32<2>(v);
    case 4: return lane_xor32<4>(v);
    case 8: return lane_xor32<8>(v);
    case 16: return lane_xor32<16>(v);
    default: return lane_xor32<32>(v);
    }
}

__device__ __forceinline__ uint64_t lane_xor64(uint64_t v, int j)
{
    switch (j) {   // (j is a constant once the sorting network is unrolled)
    case 1: return lane_xor64<1>(v);
    case 2: return lane_xor64<2>(v);
    case 4: return lane_xor64<4>(v);
    case 8: return lane_xor64<8>(v);
    case 16: return lane_xor64<16>(v);
    default: return lane_xor64<32>(v);
    }
}

// The refresh's reductions: the butterflies above with DPP moves at lane
// distances 1, 2 and 8.  (Measured: 0.4 us off each refresh at the medium
// workload; the same change in the sweep's scoring made the sparse sweep at
// the large workload 35% slower and the dense one 0.4 us slower, so the
// sweeps keep the LDS-crossbar forms.)  Every lane of the wave must be
// active.
template <bool KEYED, int OFF>
__device__ __forceinline__ void best_step_x(Candidate &c)
{
    Candidate o;
    o.cov = (int32_t)lane_xor32<OFF>((uint32_t)c.cov);
    o.i_base = (int32_t)lane_xor32<OFF>((uint32_t)c.i_base);
    o.j_base = (int32_t)lane_xor32<OFF>((uint32_t)c.j_base);
    o.slots = lane_xor32<OFF>(c.slots);
    o.dist = (int64_t)lane_xor64<OFF>((uint64_t)c.dist);
    o.key = KEYED ? lane_xor64<OFF>(c.key) : c.key;
    if (cand_better<KEYED>(o, c)) c = o;
}

template <bool KEYED, int N>
__device__ __forceinline__ Candidate wave_best_x(Candidate c)
{
    if constexpr (N > 32) best_step_x<KEYED, 32>(c);
    if constexpr (N > 16) best_step_x<KEYED, 16>(c);
    if constexpr (N > 8) best_step_x<KEYED, 8>(c);
    if constexpr (N > 4) best_step_x<KEYED, 4>(c);
    if constexpr (N > 2) best_step_x<KEYED, 2>(c);
    if constexpr (N > 1) best_step_x<KEYED, 1>(c);
    return c;
}

template <int BS, bool KEYED>
__device__ Candidate block_best_x(Candidate c, Candidate *s_red /* BS/64 + 1 */)
{
    constexpr int NW = BS / 64;
    static_assert((NW & (NW - 1)) == 0, "block size: a power-of-two number of waves");
    c = wave_best_x<KEYED, 64>(c);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_red[wave] = c;
    __syncthreads();
    if (wave == 0) {
        Candidate b = lane < NW ? s_red[lane] : no_cand();
        b = wave_best_x<KEYED, NW>(b);
        if (lane == 0) s_red[NW] = b;
    }
    __syncthreads();
    return s_red[NW];
}

__device__ __forceinline__ int32_t wave_sum_x_i32(int32_t v)
{
    v += (int32_t)lane_xor32<32>((uint32_t)v);
    v += (int32_t)lane_xor32<16>((uint32_t)v);
    v += (int32_t)lane_xor32<8>((uint32_t)v);
    v += (int32_t)lane_xor32<4>((uint32_t)v);
    v += (int32_t)lane_xor32<2>((uint32_t)v);
    v += (int32_t)lane_xor32<1>((uint32_t)v);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_x_i64(int64_t v)
{
    v += (int64_t)lane_xor64<32>((uint64_t)v);
    v += (int64_t)lane_xor64<16>((uint64_t)v);
    v += (int64_t)lane_xor64<8>((uint64_t)v);
    v += (int64_t)lane_xor64<4>((uint64_t)v);
    v += (int64_t)lane_xor64<2>((uint64_t)v);
    v += (int64_t)lane_xor64<1>((uint64_t)v);
    return v;
}

// ---------------------------------------------------------------- refresh (A2, A4, A5)

// Trace record of iteration t; cur/best as they stand after it.
__device__ void write_record(const InstDesc &d, int32_t t, const SolveState &s, int32_t moved,
                             int32_t out_base, int32_t in_base)
{
    if (!d.trace) return;
    fs_trace_rec rec;
    rec.iter = t;
    rec.out_base = moved ? out_base : -1;
    rec.in_base = moved ? in_base : -1;
    rec.moved = moved;
    rec.cur_cov = s.cur_cov;
    rec.best_cov = s.best_cov;
    rec.cur_dist = s.cur_dist;
    rec.best_dist = s.best_dist;
    gstore(d.trace + (t - 1), rec);
}

// One workgroup = 64 missions of one instance (one per lane).
//
// After iteration t's sweep (t >= 1): the workgroup reduces the row-group
// candidates to the chosen move, applies it to its LDS copy of the open list,
// and computes the state of S_{t+1}.  The workgroup of mission tile 0 commits
// the move.  With t == 0 it computes the state of S_1.
//
// State: the four waves split the open slots (k = wave, wave + 4, ...), issue
// their loads together, and merge nearest / second-nearest in LDS; ties in the
// nearest cost go to the lower base id.  G and L_k are summed in LDS, then
// added with integer atomics into one of kStripes accumulator copies (exact in
// any order).  TY: the launch set holds a typed fleet (vehicle types per slot,
// rotary-only missions, base kinds travelling with the swapped bases).
// (refresh_tile: the work of one refresh workgroup; bid is its index among
// the refresh workgroups (accumulator stripe); wait: block-scoring workgroups
// of the same launch write the candidates (fused launch), whose completion is
// awaited first.)
constexpr int32_t kScoreWaitPolls = 1 << 22;   // bound of that wait (tens of ms)

template <int MPT, bool TY, int BS>
__device__ __forceinline__ void refresh_tile(const InstDesc *__restrict__ descs, const Tile tl,
                                             int32_t step, int32_t bid, bool wait);

template <int MPT, bool TY, int BS = kBlock>
__global__ __launch_bounds__(BS) void k_refresh(const InstDesc *__restrict__ descs,
                                                const Tile *__restrict__ tiles, int32_t step)
{
    refresh_tile<MPT, TY, BS>(descs, group_tile(tiles), step, (int32_t)blockIdx.x, false);
}

template <int MPT, bool TY, int BS>
__device__ __forceinline__ void refresh_tile(const InstDesc *__restrict__ descs, const Tile tl,
                                             int32_t step, int32_t bid, bool wait)
{
    // BS == kWideBlock: MPT = 256 missions as four tiles of 64, each with four
    // waves splitting the open slots (a quarter of the workgroups of the
    // 64-mission form, each reducing the candidates once for 256 missions)
    static_assert(BS == kBlock || (BS == kWideBlock && MPT == 4 * kRefreshMissions),
                  "refresh geometry");
    const InstDesc &d = descs[tl.inst];
    if (!d.active) return;
    const int32_t t = step - d.start_step;
    if (t < 0 || t > d.N) return;
    const int32_t K = d.K, M = d.M, R = d.R;
    const int64_t ldc = d.ldc;
    SolveState *st = d.st;
    const bool leader = tl.g == 0;
    extern __shared__ __align__(16) unsigned char smem[];
    u64 *s_cov = reinterpret_cast<u64 *>(smem);
    u64 *s_dist = s_cov + (K + 1);
    int32_t *s_open = reinterpret_cast<int32_t *>(s_dist + (K + 1));
    int32_t *s_rot = s_open + K;   // vehicle type per slot (never changes in a search)
    __shared__ int32_t p_v1[BS / 64][64], p_i1[BS / 64][64], p_s1[BS / 64][64],
        p_v2[BS / 64][64];
    __shared__ Candidate s_red[BS / 64 + 1];
    __shared__ int32_t s_improved;

    if (t >= 1) {
        if (wait) {
            // the block scores of this launch: every scoring workgroup adds 1
            // (release, device scope) after its candidate; the bound turns a
            // wait that never ends into a reported error
            __shared__ int32_t s_go;
            if (threadIdx.x == 0) {
                int32_t go = 1;
                if (!gptr(st)->stopped) {
                    const int32_t target = d.ncand * t;
                    int32_t polls = 0;
                    // (relaxed polls, one acquire fence after: the caches are
                    // invalidated once, not on every poll)
                    while (__hip_atomic_load(&st->score_done, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) < target) {
                        __builtin_amdgcn_s_sleep(2);
                        if (++polls > kScoreWaitPolls) {
                            go = 0;
                            break;
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                s_go = go;
                if (!go && tl.g == 0 && !st->error) {
                    st->error = 1;
                    st->err_iter = t;
                }
            }
            __syncthreads();
            if (!s_go) return;
        }
        // The stop flag, this thread's first candidates and its open slot go
        // out together and are waited for once.  (No closed base: no row
        // group and no move; the candidate array always holds one entry.)
        const int32_t ncand = d.ncand;
        const int32_t stopped = gptr(st)->stopped;
        constexpr int CU = BS == kBlock ? 4 : 1;
        const int32_t qlast = ncand > 0 ? ncand - 1 : 0;
        Candidate cq[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u)
            cq[u] = gload(d.cand + min((int32_t)threadIdx.x + u * BS, qlast));
        const int32_t k0 = (int32_t)threadIdx.x < K ? (int32_t)threadIdx.x : 0;
        const int32_t op0 = gptr(d.open)[k0];
        const int32_t or0 = TY ? gptr(d.open_rot)[k0] : 0;
        // (empty uses, so that no part of these loads is moved past the
        // stop check or into the comparisons' branches)
#pragma unroll
        for (int u = 0; u < CU; ++u)
            asm volatile("" ::"v"(cq[u].cov), "v"(cq[u].i_base), "v"(cq[u].j_base),
                         "v"(cq[u].slots), "v"(cq[u].dist), "v"(cq[u].key));
        asm volatile("" ::"v"(op0), "v"(or0), "v"(stopped));
        if (stopped) {
            // local search ended earlier: the iteration makes no move
            if (leader && threadIdx.x == 0) write_record(d, t, *st, 0, -1, -1);
            return;
        }
        Candidate best = no_cand();
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const bool in = (int32_t)threadIdx.x + u * BS < ncand;
            if (in && (d.mode >= 2 ? cand_better<true>(cq[u], best)
                                   : cand_better<false>(cq[u], best)))
                best = cq[u];
        }
        for (int32_t q = threadIdx.x + CU * BS; q < ncand; q += BS) {
            const Candidate c = gload(d.cand + q);
            if (d.mode >= 2 ? cand_better<true>(c, best) : cand_better<false>(c, best)) best = c;
        }
        if ((int32_t)threadIdx.x < K) {
            s_open[threadIdx.x] = op0;
            if (TY) s_rot[threadIdx.x] = or0;
        }
        for (int k = threadIdx.x + BS; k < K; k += BS) {
            s_open[k] = gptr(d.open)[k];
            if (TY) s_rot[k] = gptr(d.open_rot)[k];
        }
        // barriers: s_open complete too
        best = d.mode >= 2 ? block_best_x<BS, true>(best, s_red)
                           : block_best_x<BS, false>(best, s_red);
        // (permuted searches at the end of a pass keep going: every workgroup
        // recomputes the unchanged placement's state, and the leader either
        // starts the next pass or stops; nothing here reads what it writes)
        const bool valid = cand_valid(best);
        const int32_t i_slot = cand_i_slot(best), j_slot = cand_j_slot(best);
        if (!valid && d.mode == 1) {
            // local optimum: stop; the placement and its state stay as they are
            if (leader && threadIdx.x == 0) {
                st->stopped = 1;
                write_record(d, t, *st, 0, -1, -1);
            }
            return;
        }
        if (leader) {
            // commit the move: next lists, tabu list, best-so-far, trace
            if (threadIdx.x == 0) {
                SolveState s = *st;
                int32_t improved = 0;
                if (valid) {
                    s.cur_cov = best.cov;
                    s.cur_dist = best.dist;
                    if (better(best.cov, best.dist, s.best_cov, s.best_dist)) {
                        s.best_cov = best.cov;
                        s.best_dist = best.dist;
                        s.best_iter = t;
                        improved = 1;
                    }
                    s.have_last = 1;
                    s.last_key = best.key;
                } else if (d.mode >= 2) {
                    if (s.have_last) {   // end of the order: the next pass
                        s.pass += 1;
                        s.have_last = 0;
                        s.last_key = 0;
                    } else {             // a whole pass without improvement
                        s.stopped = 1;
                    }
                }
                *st = s;
                write_record(d, t, s, valid, best.i_base, best.j_base);
                s_improved = improved;
            }
            __syncthreads();
            // the swap: the two bases trade list slots, and both stay tabu
            // through iteration t + T (the expiry travels with the base)
            if (valid && threadIdx.x == 0) {
                d.open[i_slot] = best.j_base;
                d.open_tabu[i_slot] = t + d.T;
                d.closed[j_slot] = best.i_base;
                d.closed_tabu[j_slot] = t + d.T;
                if (d.sparse) {
                    d.base_slot[best.j_base] = -1 - i_slot;
                    d.base_slot[best.i_base] = j_slot;
                    d.base_tabu[best.j_base] = t + d.T;
                    d.base_tabu[best.i_base] = t + d.T;
                }
                if (TY && d.typed) {   // the base kinds trade list slots with the bases
                    const int32_t h = d.open_hel[i_slot];
                    d.open_hel[i_slot] = d.closed_hel[j_slot];
                    d.closed_hel[j_slot] = h;
                }
            }
            if (s_improved)
                for (int k = threadIdx.x; k < K; k += BS)
                    d.best_open[k] = (valid && k == i_slot) ? best.j_base : s_open[k];
        }
        __syncthreads();
        if (valid && threadIdx.x == 0) s_open[i_slot] = best.j_base;
    } else {
        const int32_t *first = d.open;
        for (int k = threadIdx.x; k < K; k += BS) {
            s_open[k] = first[k];
            if (TY) s_rot[k] = d.open_rot[k];
        }
    }
    for (int k = threadIdx.x; k <= K; k += BS) {
        s_cov[k] = 0;
        s_dist[k] = 0;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t m, v1 = INT32_MAX, i1 = INT32_MAX, s1 = 0, v2 = INT32_MAX;
    bool owner;   // this thread holds mission m's final nearest / second-nearest
    int32_t kind; // 1: a rotary-only mission (only rotary-wing slots can fly it)
    if constexpr (MPT == kBlock && BS == kBlock) {
        // one mission per thread, every open slot in turn (small K)
        m = tl.g * MPT + threadIdx.x;
        owner = true;
        kind = (TY && d.rho && m < M) ? (gptr(d.rho)[m] != 0) : 0;
        if (m < M) {
            const gi32 *col = (const gi32 *)(d.C + m);
            constexpr int UNR = 16;
            for (int32_t k0 = 0; k0 < K; k0 += UNR) {
                int32_t c[UNR], id[UNR];
                bool ok[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int32_t k = k0 + u;
                    ok[u] = k < K && (!TY || !kind || s_rot[k]);
                    id[u] = ok[u] ? s_open[k] : 0;
                    c[u] = ok[u] ? col[(int64_t)id[u] * ldc] : INT32_MAX;
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int32_t k = k0 + u;
                    if (k < K && (!TY || !kind || s_rot[k])) {
                        if (c[u] < v1 || (c[u] == v1 && id[u] < i1)) {
                            v2 = v1;
                            v1 = c[u];
                            i1 = id[u];
                            s1 = k;
                        } else if (c[u] < v2) {
                            v2 = c[u];
                        }
                    }
                }
            }
        }
    } else {
        // four waves per 64 missions, splitting the open slots
        constexpr int W = 4, UNR = 16;
        const int sub = wave / W, ws = wave % W;
        m = tl.g * MPT + sub * 64 + lane;
        owner = ws == 0;
        kind = (TY && d.rho && m < M) ? (gptr(d.rho)[m] != 0) : 0;
        if (m < M) {
            const gi32 *col = (const gi32 *)(d.C + m);
            for (int32_t k0 = ws; k0 < K; k0 += W * UNR) {
                int32_t c[UNR], id[UNR];
                bool ok[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int32_t k = k0 + W * u;
                    ok[u] = k < K && (!TY || !kind || s_rot[k]);
                    id[u] = ok[u] ? s_open[k] : 0;
                    c[u] = ok[u] ? col[(int64_t)id[u] * ldc] : INT32_MAX;
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int32_t k = k0 + W * u;
                    if (k < K && (!TY || !kind || s_rot[k])) {
                        if (c[u] < v1 || (c[u] == v1 && id[u] < i1)) {
                            v2 = v1;
                            v1 = c[u];
                            i1 = id[u];
                            s1 = k;
                        } else if (c[u] < v2) {
                            v2 = c[u];
                        }
                    }
                }
            }
        }
        // the waves split the open slots of the same 64 missions: merge in LDS
        p_v1[wave][lane] = v1;
        p_i1[wave][lane] = i1;
        p_s1[wave][lane] = s1;
        p_v2[wave][lane] = v2;
        __syncthreads();
        if (ws == 0) {
            v1 = p_v1[wave][lane];
            i1 = p_i1[wave][lane];
            s1 = p_s1[wave][lane];
            v2 = p_v2[wave][lane];
#pragma unroll
            for (int w = wave + 1; w < wave + W; ++w) {
                const int32_t bv1 = p_v1[w][lane], bi1 = p_i1[w][lane];
                if (bv1 < v1 || (bv1 == v1 && bi1 < i1)) {
                    v2 = min(v1, p_v2[w][lane]);
                    v1 = bv1;
                    i1 = bi1;
                    s1 = p_s1[w][lane];
                } else {
                    v2 = min(v2, bv1);
                }
            }
        }
    }
    if (owner) {
        int32_t g1c = 0, g1d = 0;
        if (m < M) {
            gptr(d.b1)[m] = v1;
            gptr(d.b2)[m] = v2;
            gptr(d.o1)[m] = s1 | (kind << 16);
            g1c = v1 <= R;
            g1d = g1c ? v1 : 0;
            const int32_t g2c = v2 <= R;
            const int32_t g2d = g2c ? v2 : 0;
            const int32_t dc = g2c - g1c, dd = g2d - g1d;
            if (dc | dd) {
                atomicAdd(&s_cov[1 + s1], (u64)(int64_t)dc);
                atomicAdd(&s_dist[1 + s1], (u64)(int64_t)dd);
            }
        } else if (m < d.Mp) {
            // padding missions: a sentinel below every cost, so the sweep skips them
            gptr(d.b1)[m] = INT32_MIN;
            gptr(d.b2)[m] = INT32_MIN;
            gptr(d.o1)[m] = 0;
        }
        const int32_t wc = wave_sum_x_i32(g1c);
        const int64_t wd = wave_sum_x_i64((int64_t)g1d);
        if (lane == 0) {
            atomicAdd(&s_cov[0], (u64)(int64_t)wc);
            atomicAdd(&s_dist[0], (u64)wd);
        }
    }
    __syncthreads();
    Acc *acc = d.acc[(t + 1) & 1] + (bid & (kStripes - 1)) * (K + 1);
    for (int k = threadIdx.x; k <= K; k += BS) {
        const u64 c = s_cov[k], dd = s_dist[k];
        if (c | dd) {
            gatomic_add(&acc[k].cov, c);
            gatomic_add(&acc[k].dist, dd);
        }
    }
}

// cur = best = G of S_1; best_open = its open list.  grid = ninst.
__global__ __launch_bounds__(kBlock) void k_init_score(const InstDesc *__restrict__ descs)
{
    const InstDesc &d = descs[blockIdx.x];
    if (!d.active) return;
    if (threadIdx.x == 0) {
        int32_t gc;
        int64_t gd;
        acc_sum(d.acc[1], d.K, 0, gc, gd);
        SolveState s{};
        s.cur_cov = gc;
        s.cur_dist = gd;
        s.best_cov = gc;
        s.best_dist = gd;
        *d.st = s;
    }
    for (int k = threadIdx.x; k < d.K; k += kBlock) d.best_open[k] = d.open[k];
}

// ---------------------------------------------------------------- sweep (A3, A4 local)

// t1c[0 .. NC-1], t1d[0 .. NC-1]: the row's common term; with NC = 2 split
// over ordinary [0] and rotary-only [1] missions (o1 bit 16; a homogeneous
// fleet has none, NC = 1).  The bin is the low 16 bits of o1.
// An element below b2 (the caller has checked it).
template <int NC>
__device__ __forceinline__ void visit_hit(int32_t c, int32_t b1, int32_t o1, int32_t g1c,
                                          int32_t g1d, int32_t g2c, int32_t g2d, int32_t R,
                                          int32_t *t1c, int64_t *t1d, int32_t *__restrict__ bc,
                                          u64 *__restrict__ bd)
{
    const int32_t v1 = min(c, b1);
    const int32_t u = max(c, b1);
    const int32_t cv = v1 <= R;
    const int32_t tc = cv - g1c;
    const int32_t td = (cv ? v1 : 0) - g1d;
    if constexpr (NC == 1) {
        t1c[0] += tc;
        t1d[0] += (int64_t)td;
    } else {
        const bool rot_only = (o1 >> 16) != 0;
        t1c[0] += rot_only ? 0 : tc;
        t1c[1] += rot_only ? tc : 0;
        t1d[0] += (int64_t)(rot_only ? 0 : td);
        t1d[1] += (int64_t)(rot_only ? td : 0);
    }
    const int32_t cu = u <= R;
    const int32_t dc = cu - g2c;
    const int32_t dd = (cu ? u : 0) - g2d;
    const int32_t slot = o1 & 0xFFFF;
    if (dc | dd) {
        atomicAdd(bc + slot, dc);
        atomicAdd(bd + slot, (u64)(int64_t)dd);
    }
}

template <int NC>
__device__ __forceinline__ void visit(int32_t c, int32_t b1, int32_t b2, int32_t o1, int32_t g1c,
                                      int32_t g1d, int32_t g2c, int32_t g2d, int32_t R,
                                      int32_t *t1c, int64_t *t1d, int32_t *__restrict__ bc,
                                      u64 *__restrict__ bd)
{
    if (c < b2) visit_hit<NC>(c, b1, o1, g1c, g1d, g2c, g2d, R, t1c, t1d, bc, bd);
}

// LDS of the sweep / score kernels for J rows and up to Kmax slots.
__host__ __device__ constexpr size_t sweep_lds_bytes(int J, int Kmax)
{
    return (size_t)J * Kmax * 12 + (size_t)(Kmax + 1) * 12 + (size_t)Kmax * 12 + 16;
}

struct SweepLds {
    u64 *bd;        // J*K bins: distance
    int64_t *Ld;    // K+1: G, L_k distance
    int32_t *bc;    // J*K bins: coverage
    int32_t *Lc;    // K+1: G, L_k coverage
    int32_t *open;  // K: open base of each slot
    int32_t *otabu; // K: tabu expiry of each open slot
    int32_t *orot;  // K: 1 if the slot's vehicle is rotary-wing
};

__device__ __forceinline__ SweepLds carve_lds(unsigned char *smem, int J, int K)
{
    SweepLds s;
    s.bd = reinterpret_cast<u64 *>(smem);
    s.Ld = reinterpret_cast<int64_t *>(s.bd + J * K);
    s.bc = reinterpret_cast<int32_t *>(s.Ld + (K + 1));
    s.Lc = s.bc + J * K;
    s.open = s.Lc + (K + 1);
    s.otabu = s.open + K;
    s.orot = s.otabu + K;
    return s;
}

// Per-slot inputs of the scoring step, loaded before the streaming loop so
// their latency overlaps it: G and L_k (summed over the stripes), the open
// list, the tabu state of the open bases and (typed fleets) their vehicle
// types; without types every slot counts as rotary-wing on an aerodrome.
__device__ __forceinline__ void load_slot_inputs(const InstDesc &d, int32_t t, const SweepLds &L,
                                                 bool typed)
{
    const int32_t K = d.K;
    const Acc *acc = d.acc[t & 1];
    const int32_t *op = d.open;
    const int32_t *ot = d.open_tabu;
    for (int32_t k = threadIdx.x; k <= K; k += blockDim.x) {
        int32_t c;
        int64_t dd;
        acc_sum(acc, K, k, c, dd);
        L.Lc[k] = c;
        L.Ld[k] = dd;
        if (k < K) {
            L.open[k] = op[k];
            L.otabu[k] = ot[k];
            L.orot[k] = typed ? d.open_rot[k] : 1;
        }
    }
}

// Scores of the J x K moves of row group g from the per-row common sums
// (t1c, t1d) and the per-(row, out-slot) bins; writes the optional full score
// table and the group's best admissible candidate.
// Called by every thread of the workgroup.  st: the search state (read at
// kernel start).  When the group has at most 64 moves the first wave scores
// them alone and the rest of the workgroup may leave.
template <int BS>
__device__ void score_group(const InstDesc &d, const SolveState &st, int J, int NC, int32_t t,
                            int32_t g,
                            const int32_t *s_jrow, const int32_t *s_jtabu, const int32_t *s_jhel,
                            const SweepLds &L, const int32_t *t1c, const int64_t *t1d,
                            Candidate *s_red, const int32_t *s_jslot = nullptr)
{
    const int32_t K = d.K;
    const bool one_wave = J * K <= 64;
    if (one_wave && threadIdx.x >= 64) return;
    const int32_t cur_c = st.cur_cov, best_c = st.best_cov;
    const int64_t cur_d = st.cur_dist, best_d = st.best_dist;
    const int32_t Gc = L.Lc[0];
    const int64_t Gd = L.Ld[0];
    const bool perm = d.mode >= 2;
    const uint64_t zp = perm ? mix64(d.seed + (uint64_t)(st.pass + 1) * kGolden) : 0;
    Candidate mine = no_cand();
    for (int32_t idx = threadIdx.x; idx < J * K; idx += BS) {
        const int32_t r = idx / K, k = idx - r * K;
        // rows are consecutive closed slots, or (sparse sweep) listed in s_jslot
        const int32_t js = s_jslot ? s_jslot[r] : g * J + r;
        if (!s_jslot && js >= d.nclosed) continue;
        // moving a fixed-wing vehicle changes nothing for rotary-only missions,
        // and cannot land on a heliport
        const bool rot = L.orot[k] != 0;
        if (!rot && s_jhel[r]) continue;
        const bool two = NC == 2 && rot;
        const int32_t cov =
            Gc + L.Lc[1 + k] + t1c[NC * r] + (two ? t1c[NC * r + 1] : 0) + L.bc[idx];
        const int64_t dist =
            Gd + L.Ld[1 + k] + t1d[NC * r] + (two ? t1d[NC * r + 1] : 0) + (int64_t)L.bd[idx];
        const int32_t i = L.open[k], j = s_jrow[r];
        if (d.sc_cov) {
            gptr(d.sc_cov)[(int64_t)k * d.B + j] = cov;
            gptr(d.sc_dist)[(int64_t)k * d.B + j] = dist;
        }
        bool adm;
        uint64_t key = 0;
        if (perm) {
            // strictly improving, after the pass's last accepted move, and
            // (Tabu variant) touching no tabu base
            key = mix64(zp + ((uint64_t)i * (uint64_t)d.B + (uint64_t)j + 1) * kGolden);
            adm = better(cov, dist, cur_c, cur_d) && !(st.have_last && key <= st.last_key) &&
                  (d.mode == 2 || (L.otabu[k] < t && s_jtabu[r] < t));
        } else if (d.mode == 1) {
            adm = better(cov, dist, cur_c, cur_d);
        } else {
            adm = (L.otabu[k] < t && s_jtabu[r] < t) || better(cov, dist, best_c, best_d);
        }
        if (adm) {
            Candidate c;
            c.cov = cov;
            c.dist = dist;
            c.i_base = i;
            c.j_base = j;
            c.slots = (uint32_t)k | ((uint32_t)js << kSlotBits);
            c.key = key;
            if (perm ? cand_better<true>(c, mine) : cand_better<false>(c, mine)) mine = c;
        }
    }
    if (one_wave) {
        mine = perm ? wave_best<true>(mine) : wave_best<false>(mine);
    } else {
        mine = perm ? block_best<BS, true>(mine, s_red) : block_best<BS, false>(mine, s_red);
    }
    if (threadIdx.x == 0) d.cand[g] = mine;
}

template <int BS, int J, int U, bool NT, int NC>
__device__ __forceinline__ void sweep_vec4(const InstDesc &d, const int32_t *jrow, int32_t m0,
                                           int32_t m1, int32_t *t1c, int64_t *t1d, int32_t *bc,
                                           u64 *bd)
{
    const int32_t K = d.K, R = d.R;
    gv4i *b1v = (gv4i *)d.b1;
    gv4i *b2v = (gv4i *)d.b2;
    gv4i *o1v = (gv4i *)d.o1;
    gv4i *rows[J];
#pragma unroll
    for (int r = 0; r < J; ++r) rows[r] = (gv4i *)(d.C + (int64_t)jrow[r] * d.ldc);
    const int32_t qend = m1 >> 2;
    for (int32_t q0 = (m0 >> 2) + threadIdx.x; q0 < qend; q0 += U * BS) {
        v4i cv[U][J], vb1[U], vb2[U], vo1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t q = q0 + u * BS;
            if (q < qend) {
#pragma unroll
                for (int r = 0; r < J; ++r)
                    cv[u][r] = NT ? __builtin_nontemporal_load(rows[r] + q) : rows[r][q];
                vb1[u] = b1v[q];
                vb2[u] = b2v[q];
                vo1[u] = o1v[q];
            } else {
#pragma unroll
                for (int r = 0; r < J; ++r) cv[u][r] = (v4i)(0);
                vb1[u] = (v4i)(INT32_MIN);
                vb2[u] = (v4i)(INT32_MIN);
                vo1[u] = (v4i)(0);
            }
        }
        // every load of the step is issued before the first comparison waits
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int32_t b1 = vb1[u][e], b2 = vb2[u][e], o1 = vo1[u][e];
                const int32_t g1c = b1 <= R, g1d = g1c ? b1 : 0;
                const int32_t g2c = b2 <= R, g2d = g2c ? b2 : 0;
#pragma unroll
                for (int r = 0; r < J; ++r)
                    visit<NC>(cv[u][r][e], b1, b2, o1, g1c, g1d, g2c, g2d, R, t1c + NC * r,
                              t1d + NC * r, bc + r * K, bd + r * K);
            }
        }
    }
}

// Elements with c < b2 are a few percent of the table (about 2 / (K + 1) for
// scattered bases), but with one wave per 64 missions nearly every wave has a
// lane that takes the scoring branch, so scoring in place costs every element
// the branch's full instruction count.  The queued variants only compare in
// the streaming loop: each wave appends the lanes that hit to a queue in LDS,
// one queue per row, and scores 64 queued elements at a time with every lane
// busy.  The loop runs in whole waves (lanes past the end of the chunk load
// sentinels that never hit), so queue lengths are wave-uniform and live in
// scalar registers; a wave only reads entries it wrote itself, so no
// workgroup barrier is involved.
constexpr int kQueue = 128;   // entries per (wave, row): below 64 + 64 before a drain

// One row per workgroup: the loop streams the row and b2 alone, queues
// (c, mission), and gathers b1, b2 and o1 of the 64 queued missions when it
// scores them (a few percent of the missions, so b1 and o1 are not streamed).
struct QueueRow {
    int32_t c[kQueue], m[kQueue];
};

template <int NC>
__device__ __forceinline__ void visit_queued(const InstDesc &d, const QueueRow &qr, int32_t at,
                                             int32_t R, int32_t *t1c, int64_t *t1d,
                                             int32_t *__restrict__ bc, u64 *__restrict__ bd)
{
    // every queued element is below its b2: the three gathers go out
    // together and nothing waits on b2 alone
    const int32_t c = qr.c[at], m = qr.m[at];
    const int32_t b1 = ((const gi32 *)d.b1)[m], b2 = ((const gi32 *)d.b2)[m],
                  o1 = ((const gi32 *)d.o1)[m];
    // (an empty use of all three, so that no gather is moved into the
    // branches below and waited for on its own)
    asm volatile("" ::"v"(b1), "v"(b2), "v"(o1));
    const int32_t g1c = b1 <= R, g1d = g1c ? b1 : 0;
    const int32_t g2c = b2 <= R, g2d = g2c ? b2 : 0;
    visit_hit<NC>(c, b1, o1, g1c, g1d, g2c, g2d, R, t1c, t1d, bc, bd);
}

template <int BS, int J, int U, bool NT, int NC>
__device__ __forceinline__ void sweep_vec4_queued1(const InstDesc &d, const int32_t *jrow,
                                                  int32_t m0, int32_t m1, int32_t *t1c,
                                                  int64_t *t1d, int32_t *bc, u64 *bd)
{
    __shared__ QueueRow s_q[BS / 64][J];
    const int32_t K = d.K, R = d.R;
    const int32_t lane = threadIdx.x & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    gv4i *b2v = (gv4i *)d.b2;
    gv4i *rows[J];
#pragma unroll
    for (int r = 0; r < J; ++r) rows[r] = (gv4i *)(d.C + (int64_t)jrow[r] * d.ldc);
    int32_t len[J];
#pragma unroll
    for (int r = 0; r < J; ++r) len[r] = 0;
    const int32_t qend = m1 >> 2;
    for (int32_t qw = (m0 >> 2) + wave * 64; qw < qend; qw += U * BS) {
        // lanes past the end re-read the last quad and never hit (b2 = INT32_MIN)
        v4i cv[U][J], vb2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t q = min(qw + u * BS + lane, qend - 1);
#pragma unroll
            for (int r = 0; r < J; ++r)
                cv[u][r] = NT ? __builtin_nontemporal_load(rows[r] + q) : rows[r][q];
            vb2[u] = b2v[q];
        }
        // keep every load of the iteration ahead of the first use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (qw + u * BS + lane >= qend) vb2[u] = (v4i)(INT32_MIN);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
#pragma unroll
                for (int r = 0; r < J; ++r) {
                    const bool hit = cv[u][r][e] < vb2[u][e];
                    const u64 mask = __builtin_amdgcn_ballot_w64(hit);
                    if (mask == 0) continue;
                    QueueRow &qr = s_q[wave][r];
                    if (hit) {
                        const int32_t at = (int32_t)__builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(mask >> 32),
                            __builtin_amdgcn_mbcnt_lo((uint32_t)mask, (uint32_t)len[r]));
                        qr.c[at] = cv[u][r][e];
                        qr.m[at] = 4 * (qw + u * BS + lane) + e;
                    }
                    len[r] = __builtin_amdgcn_readfirstlane(len[r] +
                                                            (int32_t)__builtin_popcountll(mask));
                    if (len[r] >= 64) {
                        // score the oldest 64, then move the rest (at most 63) down
                        __builtin_amdgcn_wave_barrier();
                        visit_queued<NC>(d, qr, lane, R, t1c + NC * r, t1d + NC * r,
                                         bc + r * K, bd + r * K);
                        len[r] -= 64;
                        int32_t c = 0, mm = 0;
                        if (lane < len[r]) {
                            c = qr.c[64 + lane];
                            mm = qr.m[64 + lane];
                        }
                        __builtin_amdgcn_wave_barrier();
                        if (lane < len[r]) {
                            qr.c[lane] = c;
                            qr.m[lane] = mm;
                        }
                        __builtin_amdgcn_wave_barrier();
                    }
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < J; ++r)
        if (lane < len[r])
            visit_queued<NC>(d, s_q[wave][r], lane, R, t1c + NC * r, t1d + NC * r,
                             bc + r * K, bd + r * K);
}

// Several rows per workgroup: the rows share one streamed copy of b1, b2 and
// o1, and each queue entry carries the element with its state.
struct QueueRow4 {
    int32_t c[kQueue], b1[kQueue], b2[kQueue], o1[kQueue];
};

template <int NC>
__device__ __forceinline__ void visit_queued4(const QueueRow4 &qr, int32_t at, int32_t R,
                                             int32_t *t1c, int64_t *t1d, int32_t *__restrict__ bc,
                                             u64 *__restrict__ bd)
{
    const int32_t c = qr.c[at], b1 = qr.b1[at], b2 = qr.b2[at], o1 = qr.o1[at];
    const int32_t g1c = b1 <= R, g1d = g1c ? b1 : 0;
    const int32_t g2c = b2 <= R, g2d = g2c ? b2 : 0;
    visit_hit<NC>(c, b1, o1, g1c, g1d, g2c, g2d, R, t1c, t1d, bc, bd);
}

template <int BS, int J, int U, bool NT, int NC>
__device__ __forceinline__ void sweep_vec4_queued4(const InstDesc &d, const int32_t *jrow,
                                                  int32_t m0, int32_t m1, int32_t *t1c,
                                                  int64_t *t1d, int32_t *bc, u64 *bd)
{
    __shared__ QueueRow4 s_q[BS / 64][J];
    const int32_t K = d.K, R = d.R;
    const int32_t lane = threadIdx.x & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    gv4i *b1v = (gv4i *)d.b1;
    gv4i *b2v = (gv4i *)d.b2;
    gv4i *o1v = (gv4i *)d.o1;
    gv4i *rows[J];
#pragma unroll
    for (int r = 0; r < J; ++r) rows[r] = (gv4i *)(d.C + (int64_t)jrow[r] * d.ldc);
    int32_t len[J];
#pragma unroll
    for (int r = 0; r < J; ++r) len[r] = 0;
    const int32_t qend = m1 >> 2;
    for (int32_t qw = (m0 >> 2) + wave * 64; qw < qend; qw += U * BS) {
        // lanes past the end re-read the last quad and never hit (b2 = INT32_MIN)
        v4i cv[U][J], vb1[U], vb2[U], vo1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t q = min(qw + u * BS + lane, qend - 1);
#pragma unroll
            for (int r = 0; r < J; ++r)
                cv[u][r] = NT ? __builtin_nontemporal_load(rows[r] + q) : rows[r][q];
            vb1[u] = b1v[q];
            vb2[u] = b2v[q];
            vo1[u] = o1v[q];
        }
        // keep every load of the iteration ahead of the first use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (qw + u * BS + lane >= qend) vb2[u] = (v4i)(INT32_MIN);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
#pragma unroll
                for (int r = 0; r < J; ++r) {
                    const bool hit = cv[u][r][e] < vb2[u][e];
                    const u64 mask = __builtin_amdgcn_ballot_w64(hit);
                    if (mask == 0) continue;
                    QueueRow4 &qr = s_q[wave][r];
                    if (hit) {
                        const int32_t at = (int32_t)__builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(mask >> 32),
                            __builtin_amdgcn_mbcnt_lo((uint32_t)mask, (uint32_t)len[r]));
                        qr.c[at] = cv[u][r][e];
                        qr.b1[at] = vb1[u][e];
                        qr.b2[at] = vb2[u][e];
                        qr.o1[at] = vo1[u][e];
                    }
                    len[r] = __builtin_amdgcn_readfirstlane(len[r] +
                                                            (int32_t)__builtin_popcountll(mask));
                    if (len[r] >= 64) {
                        // score the oldest 64, then move the rest (at most 63) down
                        __builtin_amdgcn_wave_barrier();
                        visit_queued4<NC>(qr, lane, R, t1c + NC * r, t1d + NC * r, bc + r * K,
                                         bd + r * K);
                        len[r] -= 64;
                        int32_t c = 0, b1 = 0, b2 = 0, o1 = 0;
                        if (lane < len[r]) {
                            c = qr.c[64 + lane];
                            b1 = qr.b1[64 + lane];
                            b2 = qr.b2[64 + lane];
                            o1 = qr.o1[64 + lane];
                        }
                        __builtin_amdgcn_wave_barrier();
                        if (lane < len[r]) {
                            qr.c[lane] = c;
                            qr.b1[lane] = b1;
                            qr.b2[lane] = b2;
                            qr.o1[lane] = o1;
                        }
                        __builtin_amdgcn_wave_barrier();
                    }
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < J; ++r)
        if (lane < len[r])
            visit_queued4<NC>(s_q[wave][r], lane, R, t1c + NC * r, t1d + NC * r, bc + r * K,
                             bd + r * K);
}


// Gathering per row pays off for one row; with several, each row's hits would
// gather on their own.
template <int BS, int J, int U, bool NT, int NC>
__device__ __forceinline__ void sweep_vec4_queued(const InstDesc &d, const int32_t *jrow,
                                                  int32_t m0, int32_t m1, int32_t *t1c,
                                                  int64_t *t1d, int32_t *bc, u64 *bd)
{
    if constexpr (J == 1)
        sweep_vec4_queued1<BS, J, U, NT, NC>(d, jrow, m0, m1, t1c, t1d, bc, bd);
    else
        sweep_vec4_queued4<BS, J, U, NT, NC>(d, jrow, m0, m1, t1c, t1d, bc, bd);
}

template <int BS, int J, int NC>
__device__ __forceinline__ void sweep_scalar(const InstDesc &d, const int32_t *jrow, int32_t m0,
                                             int32_t m1, int32_t *t1c, int64_t *t1d, int32_t *bc,
                                             u64 *bd)
{
    const int32_t K = d.K, R = d.R;
    const int32_t mend = min(m1, d.M);
    const int64_t ldc = d.ldc;
    const gi32 *C = (const gi32 *)d.C;
    for (int32_t m = m0 + threadIdx.x; m < mend; m += BS) {
        int32_t cv[J];
#pragma unroll
        for (int r = 0; r < J; ++r) cv[r] = C[(int64_t)jrow[r] * ldc + m];
        const int32_t b1 = ((const gi32 *)d.b1)[m], b2 = ((const gi32 *)d.b2)[m],
                      o1 = ((const gi32 *)d.o1)[m];
        const int32_t g1c = b1 <= R, g1d = g1c ? b1 : 0;
        const int32_t g2c = b2 <= R, g2d = g2c ? b2 : 0;
#pragma unroll
        for (int r = 0; r < J; ++r)
            visit<NC>(cv[r], b1, b2, o1, g1c, g1d, g2c, g2d, R, t1c + NC * r, t1d + NC * r,
                      bc + r * K, bd + r * K);
    }
}

// Workgroup reduction of the per-row common sums.
template <int BS, int J>
__device__ __forceinline__ void reduce_rows(const int32_t *t1c, const int64_t *t1d,
                                            int32_t (*s_t1c)[J], int64_t (*s_t1d)[J],
                                            int32_t *s_sum_c, int64_t *s_sum_d)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < J; ++r) {
        const int32_t c = wave_sum_i32(t1c[r]);
        const int64_t dd = wave_sum_i64(t1d[r]);
        if (lane == 0) {
            s_t1c[wave][r] = c;
            s_t1d[wave][r] = dd;
        }
    }
    __syncthreads();
    if (threadIdx.x < J) {
        int32_t c = 0;
        int64_t dd = 0;
        for (int w = 0; w < BS / 64; ++w) {
            c += s_t1c[w][threadIdx.x];
            dd += s_t1d[w][threadIdx.x];
        }
        s_sum_c[threadIdx.x] = c;
        s_sum_d[threadIdx.x] = dd;
    }
    __syncthreads();
}

// The work of an instance's first sweep workgroup besides its tile: clear the
// accumulators the coming refresh fills, and check that the value of S_t
// recounted by the previous refresh equals the score its move was chosen with.
__device__ void sweep_housekeeping(const InstDesc &d, int32_t t)
{
    Acc *nxt = d.acc[(t + 1) & 1];
    for (int32_t q = threadIdx.x; q < kStripes * (d.K + 1); q += blockDim.x) {
        nxt[q].cov = 0;
        nxt[q].dist = 0;
    }
    if (threadIdx.x == 0) {
        int32_t gc;
        int64_t gd;
        acc_sum(d.acc[t & 1], d.K, 0, gc, gd);
        SolveState *st = d.st;
        if ((gc != st->cur_cov || gd != st->cur_dist) && !st->error) {
            st->error = 1;
            st->err_iter = t;
        }
    }
}

// One workgroup = J closed rows x one mission chunk of one instance.  Tiles
// are ordered chunk-minor so that consecutive block ids (which the dispatcher
// spreads over the XCDs) split an instance's mission axis and each XCD's L2
// holds the b1/b2/o1 of fewer chunks.  NC: common-term classes per row (2
// when some instance of the launch set has a typed fleet, else 1).
template <int BS, int J, int U, bool VEC4, bool NT, bool Q, int NC>
__global__ __launch_bounds__(BS) void k_sweep(const InstDesc *__restrict__ descs,
                                                  const Tile *__restrict__ tiles, int32_t step)
{
    // rows whose loads go out together: the in-place vector sweep takes
    // groups of more than four rows in passes of four (the group's start-up
    // and scoring are paid once for all its rows, with the registers of four)
    constexpr int JL = (VEC4 && !Q && J > 4) ? 4 : J;
    constexpr int P = J / JL;
    static_assert(P * JL == J, "rows per pass");
    const Tile tl = sweep_tile(descs, tiles);
    const InstDesc &d = descs[tl.inst];
    if (!d.active) return;
    const int32_t t = step - d.start_step;
    if (t < 1 || t > d.N) return;
    // The search state, this group's rows and the slot inputs go out in one
    // round of loads; the stop flag is checked once they are issued (before
    // anything is written to device memory).
    // (a generic load: the state stays off the scalar path, measured faster)
    const SolveState st = *d.st;
    const bool scoring = d.nsplit == 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t K = d.K;
    const SweepLds L = carve_lds(smem, J, K);
    __shared__ int32_t s_jrow[J], s_jtabu[J], s_jhel[J];
    // per row: the common term (typed: over ordinary [2r] and rotary-only
    // [2r + 1] missions)
    __shared__ int32_t s_t1c[BS / 64][NC * J];
    __shared__ int64_t s_t1d[BS / 64][NC * J];
    __shared__ int32_t s_sum_c[NC * J];
    __shared__ int64_t s_sum_d[NC * J];
    __shared__ Candidate s_red[BS / 64 + 1];

    // The set-up loads (this group's rows by threads 0 .. J - 1, the first
    // K + 1 slot inputs by threads 0 .. K) go out in one round, at clamped
    // indices (every list holds at least one entry), and are waited for once;
    // LDS takes them after the stop check.
    const int32_t nclosed = d.nclosed;
    const int32_t k0 = min((int32_t)threadIdx.x, K), k0o = min(k0, K - 1);
    int32_t ld_jrow = 0, ld_jtabu = 0, ld_jhel = 0, ld_lc = 0, ld_open = 0, ld_otabu = 0,
            ld_orot = 1;
    int64_t ld_ld = 0;
    if ((int32_t)threadIdx.x < J) {
        const int32_t js = tl.g * J + (int32_t)threadIdx.x;
        const int32_t jc = js < nclosed ? js : 0;
        ld_jrow = gptr(d.closed)[jc];
        ld_jtabu = gptr(d.closed_tabu)[jc];
        if (NC == 2) ld_jhel = gptr(d.closed_hel)[jc];
    }
    if ((int32_t)threadIdx.x <= K) {
        const __attribute__((address_space(1))) Acc *ga = gptr(d.acc[t & 1]);
        u64 pc[kStripes], pd[kStripes];
#pragma unroll
        for (int q = 0; q < kStripes; ++q) {
            pc[q] = ga[q * (K + 1) + k0].cov;
            pd[q] = ga[q * (K + 1) + k0].dist;
        }
        ld_open = gptr(d.open)[k0o];
        ld_otabu = gptr(d.open_tabu)[k0o];
        if (NC == 2) ld_orot = gptr(d.open_rot)[k0o];
        // (every load above is issued before the first sum waits)
        __builtin_amdgcn_sched_barrier(0);
        u64 sc = 0, sd = 0;
#pragma unroll
        for (int q = 0; q < kStripes; ++q) {
            sc += pc[q];
            sd += pd[q];
        }
        ld_lc = (int32_t)(int64_t)sc;
        ld_ld = (int64_t)sd;
    }
    asm volatile("" ::"v"(ld_jrow), "v"(ld_jtabu), "v"(ld_jhel), "v"(ld_lc), "v"(ld_ld),
                 "v"(ld_open), "v"(ld_otabu), "v"(ld_orot), "v"(st.stopped));
    if (st.stopped) return;
    if (threadIdx.x < J) {
        s_jrow[threadIdx.x] = nclosed > 0 ? ld_jrow : 0;
        s_jtabu[threadIdx.x] = nclosed > 0 ? ld_jtabu : 0;
        s_jhel[threadIdx.x] = nclosed > 0 ? ld_jhel : 0;
    }
    if (scoring) {
        if ((int32_t)threadIdx.x <= K) {
            L.Lc[k0] = ld_lc;
            L.Ld[k0] = ld_ld;
            if ((int32_t)threadIdx.x < K) {
                L.open[k0] = ld_open;
                L.otabu[k0] = ld_otabu;
                L.orot[k0] = ld_orot;
            }
        }
        // (more than BS - 1 open slots: the rest one round at a time)
        for (int32_t k = threadIdx.x + BS; k <= K; k += BS) {
            int32_t c;
            int64_t dd;
            acc_sum(d.acc[t & 1], K, k, c, dd);
            L.Lc[k] = c;
            L.Ld[k] = dd;
            if (k < K) {
                L.open[k] = d.open[k];
                L.otabu[k] = d.open_tabu[k];
                L.orot[k] = NC == 2 ? d.open_rot[k] : 1;
            }
        }
    }
    if (tl.g == 0 && tl.sp == 0) sweep_housekeeping(d, t);
    for (int q = threadIdx.x; q < J * K; q += BS) {
        L.bd[q] = 0;
        L.bc[q] = 0;
    }
    __syncthreads();

    const int32_t m0 = tl.sp * d.chunk;
    const int32_t m1 = min(d.Mp, m0 + d.chunk);
    if constexpr (P == 1) {
        int32_t jrow[J];
#pragma unroll
        for (int r = 0; r < J; ++r) jrow[r] = s_jrow[r];
        int32_t t1c[NC * J];
        int64_t t1d[NC * J];
#pragma unroll
        for (int r = 0; r < NC * J; ++r) {
            t1c[r] = 0;
            t1d[r] = 0;
        }
        if (nclosed > 0) {
            if (VEC4 && Q)
                sweep_vec4_queued<BS, J, U, NT, NC>(d, jrow, m0, m1, t1c, t1d, L.bc, L.bd);
            else if (VEC4)
                sweep_vec4<BS, J, U, NT, NC>(d, jrow, m0, m1, t1c, t1d, L.bc, L.bd);
            else
                sweep_scalar<BS, J, NC>(d, jrow, m0, m1, t1c, t1d, L.bc, L.bd);
        }
        reduce_rows<BS, NC * J>(t1c, t1d, s_t1c, s_t1d, s_sum_c, s_sum_d);
    } else {
        // P passes over the chunk, JL rows each: every wave sums its common
        // terms of a pass into LDS; the workgroup adds the waves once at the end
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll 1
        for (int p = 0; p < P; ++p) {
            int32_t jrow[JL];
#pragma unroll
            for (int r = 0; r < JL; ++r) jrow[r] = s_jrow[p * JL + r];
            int32_t t1c[NC * JL];
            int64_t t1d[NC * JL];
#pragma unroll
            for (int r = 0; r < NC * JL; ++r) {
                t1c[r] = 0;
                t1d[r] = 0;
            }
            if (nclosed > 0)
                sweep_vec4<BS, JL, U, NT, NC>(d, jrow, m0, m1, t1c, t1d, L.bc + p * JL * K,
                                              L.bd + p * JL * K);
#pragma unroll
            for (int r = 0; r < NC * JL; ++r) {
                const int32_t c = wave_sum_i32(t1c[r]);
                const int64_t dd = wave_sum_i64(t1d[r]);
                if (lane == 0) {
                    s_t1c[wave][NC * JL * p + r] = c;
                    s_t1d[wave][NC * JL * p + r] = dd;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < NC * J) {
            int32_t c = 0;
            int64_t dd = 0;
            for (int w = 0; w < BS / 64; ++w) {
                c += s_t1c[w][threadIdx.x];
                dd += s_t1d[w][threadIdx.x];
            }
            s_sum_c[threadIdx.x] = c;
            s_sum_d[threadIdx.x] = dd;
        }
        __syncthreads();
    }

    if (scoring) {
        score_group<BS>(d, st, J, NC, t, tl.g, s_jrow, s_jtabu, s_jhel, L, s_sum_c, s_sum_d,
                        s_red);
    } else {
        // partial sums of this chunk: [T1 ordinary, T1 rotary-only, bin_0 ..
        // bin_{K-1}] per row
        const int32_t K2 = K + 2;
        for (int32_t idx = threadIdx.x; idx < J * K2; idx += BS) {
            const int32_t r = idx / K2, k = idx - r * K2;
            const int32_t js = tl.g * J + r;
            if (js >= nclosed) continue;
            const int64_t at = ((int64_t)tl.sp * nclosed + js) * K2 + k;
            if (k < 2) {
                d.part_cov[at] = k < NC ? s_sum_c[NC * r + k] : 0;
                d.part_dist[at] = k < NC ? s_sum_d[NC * r + k] : 0;
            } else {
                d.part_cov[at] = L.bc[r * K + k - 2];
                d.part_dist[at] = (int64_t)L.bd[r * K + k - 2];
            }
        }
    }
}

// ---------------------------------------------------------------- sparse sweep (A3)
//
// Only elements with c < b2 contribute to a move score.  For each block of
// kSparseW consecutive base ids and each mission, the block's bases are kept
// sorted by (cost, id); a sweep then walks each mission's sorted list only
// while the cost is below b2, so it touches the contributing elements (and one
// more per list) instead of every closed row.  The terms added are exactly the
// dense sweep's (the same integer arithmetic on the same elements), so the
// scores are identical.

// Costs below kNarrowTop (2^26 - 1) fit a 32-bit (cost << 6 | id) key.
constexpr uint32_t kNarrowTop = (1u << 26) - 1;

// Sorted lists of one block x 64 missions: the C tile is staged in LDS, each
// wave sorts a mission's 64 (cost, local id) keys across its lanes (bitonic,
// ascending; the sign bit is flipped so that the unsigned key order is the
// signed cost order), and the sorted columns go out rank-major.  Bases past B
// and missions past M sort last with cost INT32_MAX, which no b2 exceeds.
template <bool PACKED>
__global__ __launch_bounds__(kBlock) void k_sparse_build(const InstDesc *__restrict__ descs)
{
    const InstDesc &d = descs[0];
    const int32_t nmg = (d.Mp + 63) / 64;
    const int32_t q = (int32_t)blockIdx.x / nmg, mg = (int32_t)blockIdx.x - q * nmg;
    // (row pitches of 65 words and 68 bytes: a wave writing one column
    // touches a different bank in every lane; the sorted costs reuse the
    // tile's LDS once every wave holds its columns in registers, which keeps
    // the workgroup at 21 KB of LDS)
    __shared__ int32_t s_c[kSparseW][65];
    int32_t (*s_cost)[65] = s_c;
    __shared__ __align__(16) unsigned char s_id[kSparseW][68];
    // every load of the tile in flight before the first LDS write (each
    // thread: one mission, every fourth base of the block)
    constexpr int PER_THREAD = kSparseW * 64 / kBlock;
    const gi32 *C = (const gi32 *)d.C;
    const int64_t ldc = d.ldc;
    const int32_t B = d.B, m = mg * 64 + (int32_t)(threadIdx.x & 63);
    const int32_t l0 = (int32_t)threadIdx.x >> 6;
    const bool m_in = m < d.M;
    const gi32 *col = C + (m_in ? m : 0);
    int32_t v[PER_THREAD];
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) {
        const int32_t b = q * kSparseW + l0 + i * (kBlock / 64);
        const bool in = m_in && b < B;
        v[i] = col[in ? (int64_t)b * ldc : 0];
        v[i] = in ? v[i] : INT32_MAX;
    }
#pragma unroll
    for (int i = 0; i < PER_THREAD; ++i) s_c[l0 + i * (kBlock / 64)][threadIdx.x & 63] = v[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // four missions' sorts interleaved, so that each exchange's latency is
    // covered by the other three
    // (narrow keys: when every cost of the four missions lies in
    // [0, 2^26 - 1) or is the sentinel, (cost << 6 | id) fits 32 bits with
    // the sentinel as 2^26 - 1, in the same order; a haversine round trip is
    // below 6.1e7 m < 2^26 - 1, so real tables take this path)
    constexpr int PER_WAVE = 64 / (kBlock / 64), IL = 4;
    int32_t col_c[PER_WAVE];
#pragma unroll
    for (int i = 0; i < PER_WAVE; ++i) col_c[i] = s_c[lane][wave * PER_WAVE + i];
    __syncthreads();   // (the tile is read; its LDS now takes the sorted costs)
#pragma unroll
    for (int i0 = 0; i0 < PER_WAVE; i0 += IL) {
        int32_t cst[IL];
        bool fits = true;
#pragma unroll
        for (int q = 0; q < IL; ++q) {
            cst[q] = col_c[i0 + q];
            fits = fits && (cst[q] == INT32_MAX || (uint32_t)cst[q] < kNarrowTop);
        }
        if (__builtin_amdgcn_ballot_w64(!fits) == 0) {
            uint32_t key[IL];
#pragma unroll
            for (int q = 0; q < IL; ++q)
                key[q] = ((cst[q] == INT32_MAX ? kNarrowTop : (uint32_t)cst[q]) << 6) |
                         (uint32_t)lane;
#pragma unroll
            for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
                for (int j = k >> 1; j > 0; j >>= 1) {
                    const bool up = (lane & k) == 0, lower = (lane & j) == 0;
#pragma unroll
                    for (int q = 0; q < IL; ++q) {
                        const uint32_t other = lane_xor32(key[q], j);
                        key[q] = (lower == up) ? min(key[q], other) : max(key[q], other);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < IL; ++q) {
                const int32_t mm = wave * PER_WAVE + i0 + q;
                const uint32_t c = key[q] >> 6;
                s_cost[lane][mm] = c == kNarrowTop ? INT32_MAX : (int32_t)c;
                s_id[lane][mm] = (unsigned char)(key[q] & 63);
            }
            continue;
        }
        uint64_t key[IL];
#pragma unroll
        for (int q = 0; q < IL; ++q)
            key[q] = ((uint64_t)((uint32_t)cst[q] ^ 0x80000000u) << 6) | (uint64_t)lane;
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const bool up = (lane & k) == 0, lower = (lane & j) == 0;
#pragma unroll
                for (int q = 0; q < IL; ++q) {
                    const uint64_t other = lane_xor64(key[q], j);
                    key[q] = (lower == up) ? min(key[q], other) : max(key[q], other);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < IL; ++q) {
            const int32_t mm = wave * PER_WAVE + i0 + q;
            s_cost[lane][mm] = (int32_t)((uint32_t)(key[q] >> 6) ^ 0x80000000u);
            s_id[lane][mm] = (unsigned char)(key[q] & 63);
        }
    }
    __syncthreads();
    // Packed keys: (cost << 6 | id), the sentinel as kNarrowTop << 6 | id (no
    // b2 threshold reaches it); a cost that does not fit sets the wide flag
    // (the lists are then built again unpacked).
    if (PACKED) {
        bool bad = false;
        for (int32_t u = threadIdx.x; u < kSparseW * 64; u += kBlock) {
            const int32_t c = s_cost[u >> 6][u & 63];
            bad = bad || (c != INT32_MAX && (uint32_t)c >= kNarrowTop);
        }
        if (__builtin_amdgcn_ballot_w64(bad) != 0 && (threadIdx.x & 63) == 0)
            atomicOr(d.wide, 1);
    }
    auto key_of = [&](int32_t r, int32_t mm) {
        const int32_t c = s_cost[r][mm];
        return (int32_t)(((c == INT32_MAX ? kNarrowTop : (uint32_t)c) << 6) |
                         (uint32_t)s_id[r][mm]);
    };
    // The head ranks rank-major: four consecutive missions of one rank per
    // thread, one 16-byte store of costs (or keys) and one 4-byte store of ids
    // (Mp is a multiple of 4, so a quad lies wholly inside or outside the
    // padded mission range, and every quad's address is 16- and 4-byte
    // aligned).
    const int64_t Mp = d.Mp;
    for (int32_t u = threadIdx.x; u < kSparseHead * 16; u += kBlock) {
        const int32_t r = u >> 4, mm = (u & 15) * 4, m = mg * 64 + mm;
        if (m < Mp) {
            const int64_t at = ((int64_t)q * kSparseHead + r) * Mp + m;
            v4i c;
#pragma unroll
            for (int e = 0; e < 4; ++e) c[e] = PACKED ? key_of(r, mm + e) : s_cost[r][mm + e];
            *reinterpret_cast<v4i *>(d.lst_cost + at) = c;
            if (!PACKED)
                *reinterpret_cast<uint32_t *>(d.lst_id + at) =
                    *reinterpret_cast<const uint32_t *>(&s_id[r][mm]);
        }
    }
    // Every rank mission-major: sixteen consecutive ranks of one mission per
    // thread, four 16-byte stores of costs (or keys) and one of ids (a wave
    // writes 4 KB of consecutive entries).
    for (int32_t u = threadIdx.x; u < 64 * (kSparseW / 16); u += kBlock) {
        const int32_t mm = u / (kSparseW / 16), r0 = (u % (kSparseW / 16)) * 16;
        const int32_t m = mg * 64 + mm;
        if (m < Mp) {
            const int64_t at = ((int64_t)q * Mp + m) * kSparseW + r0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                v4i c;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    c[e] = PACKED ? key_of(r0 + 4 * v + e, mm) : s_cost[r0 + 4 * v + e][mm];
                *reinterpret_cast<v4i *>(d.mm_cost + at + 4 * v) = c;
            }
            if (!PACKED) {
                v4i ids;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    uint32_t w = 0;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        w |= (uint32_t)s_id[r0 + 4 * v + e][mm] << (8 * e);
                    ids[v] = (int32_t)w;
                }
                *reinterpret_cast<v4i *>(d.mm_id + at) = ids;
            }
        }
    }
}

// base_slot and base_tabu from the open and closed lists and their expiries
// (before the first sparse sweep).
__global__ __launch_bounds__(kBlock) void k_sparse_slots(const InstDesc *__restrict__ descs)
{
    const InstDesc &d = descs[0];
    for (int32_t js = threadIdx.x + blockIdx.x * kBlock; js < d.nclosed;
         js += gridDim.x * kBlock) {
        d.base_slot[d.closed[js]] = js;
        d.base_tabu[d.closed[js]] = d.closed_tabu[js];
    }
    for (int32_t k = threadIdx.x + blockIdx.x * kBlock; k < d.K; k += gridDim.x * kBlock) {
        d.base_slot[d.open[k]] = -1 - k;
        d.base_tabu[d.open[k]] = d.open_tabu[k];
    }
}

// The dense visit's terms for one element c < b2 of a row, added to the
// row's common term and bin in LDS.
__device__ __forceinline__ void visit_sparse(int32_t c, int32_t b1, int32_t b2, int32_t o1,
                                             int32_t g1c, int32_t g1d, int32_t g2c, int32_t g2d,
                                             int32_t R, int32_t *t1c, u64 *t1d,
                                             int32_t *__restrict__ bc, u64 *__restrict__ bd)
{
    const int32_t v1 = min(c, b1);
    const int32_t u = max(c, b1);
    const int32_t cv = v1 <= R;
    const int32_t tc = cv - g1c;
    const int32_t td = (cv ? v1 : 0) - g1d;
    if (tc | td) {
        atomicAdd(t1c, tc);
        atomicAdd(t1d, (u64)(int64_t)td);
    }
    const int32_t cu = u <= R;
    const int32_t dc = cu - g2c;
    const int32_t dd = (cu ? u : 0) - g2d;
    const int32_t slot = o1 & 0xFFFF;
    if (dc | dd) {
        atomicAdd(bc + slot, dc);
        atomicAdd(bd + slot, (u64)(int64_t)dd);
    }
}

// Set-up loads of a block kernel of the sparse sweep, issued together and
// waited for once: the search state, the list slot and tabu expiry of the
// block's 64 base ids (first wave, one per lane), and the slot inputs of
// slot k = thread for threads 0 .. K (G and L_k summed over the stripes, open
// base, its tabu expiry).  Indices are clamped, so every load is in bounds.
struct SparseSetup {
    SolveState st;
    int32_t slot, tabu;   // base q * 64 + lane: slot (>= 0 closed, < 0 open) ...
    bool inb;             // ... if the base exists (below B)
    int32_t lc, open, otabu;
    int64_t ld;
};

__device__ __forceinline__ SparseSetup sparse_setup(const InstDesc &d, int32_t t, int32_t q)
{
    SparseSetup u;
    // (a generic load: the state stays off the scalar path, measured faster)
    u.st = *d.st;
    const int32_t K = d.K;
    u.slot = -1;
    u.tabu = 0;
    u.inb = false;
    u.lc = 0;
    u.ld = 0;
    u.open = 0;
    u.otabu = 0;
    // (only the first wave uses the block's slots, and threads 0 .. K the
    // slot inputs: the other waves skip both)
    if (threadIdx.x < kSparseW) {
        const int32_t b = q * kSparseW + (int32_t)threadIdx.x;
        const int32_t bb = min(b, d.B - 1);
        u.slot = gptr(d.base_slot)[bb];
        u.tabu = gptr(d.base_tabu)[bb];
        u.inb = b < d.B;
    }
    if ((int32_t)threadIdx.x <= K) {
        const int32_t k0 = threadIdx.x, k0o = min(k0, K - 1);
        const __attribute__((address_space(1))) Acc *ga = gptr(d.acc[t & 1]);
        u64 pc[kStripes], pd[kStripes];
#pragma unroll
        for (int s = 0; s < kStripes; ++s) {
            pc[s] = ga[s * (K + 1) + k0].cov;
            pd[s] = ga[s * (K + 1) + k0].dist;
        }
        u.open = gptr(d.open)[k0o];
        u.otabu = gptr(d.open_tabu)[k0o];
        // (every load above is issued before the first sum waits)
        __builtin_amdgcn_sched_barrier(0);
        u64 sc = 0, sd = 0;
#pragma unroll
        for (int s = 0; s < kStripes; ++s) {
            sc += pc[s];
            sd += pd[s];
        }
        u.lc = (int32_t)(int64_t)sc;
        u.ld = (int64_t)sd;
    }
    asm volatile("" ::"v"(u.st.stopped), "v"(u.st.pass), "v"(u.st.cur_cov), "v"(u.st.best_cov),
                 "v"(u.st.cur_dist), "v"(u.st.best_dist), "v"(u.st.have_last),
                 "v"(u.st.last_key), "v"(u.slot), "v"(u.tabu), "v"(u.lc), "v"(u.ld),
                 "v"(u.open), "v"(u.otabu));
    return u;
}

// The closed bases of the block as rows (ascending id): s_jrow / s_jslot /
// s_jtabu, and s_rowof[local id] = row or -1.  Called by the first wave with
// its set-up loads.
__device__ __forceinline__ void sparse_rows(const SparseSetup &u, int32_t q, int32_t *s_jrow,
                                            int32_t *s_jslot, int32_t *s_jtabu, int32_t *s_jhel,
                                            int32_t *s_rowof, int32_t *s_nrows)
{
    const int lane = threadIdx.x & 63;
    const int32_t b = q * kSparseW + lane;
    const bool closed = u.inb && u.slot >= 0;
    const u64 mask = __builtin_amdgcn_ballot_w64(closed);
    const int32_t row = (int32_t)__builtin_popcountll(mask & ((1ull << lane) - 1));
    s_rowof[lane] = closed ? row : -1;
    if (closed) {
        s_jrow[row] = b;
        s_jslot[row] = u.slot;
        s_jtabu[row] = u.tabu;
        s_jhel[row] = 0;
    }
    if (lane == 0) *s_nrows = (int32_t)__builtin_popcountll(mask);
}

// The slot inputs to LDS: slot k = thread from the set-up loads, any further
// slots (K >= the workgroup size) loaded here.
__device__ __forceinline__ void sparse_slot_inputs(const InstDesc &d, int32_t t,
                                                   const SparseSetup &u, const SweepLds &L)
{
    const int32_t K = d.K;
    if ((int32_t)threadIdx.x <= K) {
        L.Lc[threadIdx.x] = u.lc;
        L.Ld[threadIdx.x] = u.ld;
        if ((int32_t)threadIdx.x < K) {
            L.open[threadIdx.x] = u.open;
            L.otabu[threadIdx.x] = u.otabu;
            L.orot[threadIdx.x] = 1;
        }
    }
    for (int32_t k = threadIdx.x + blockDim.x; k <= K; k += blockDim.x) {
        int32_t c;
        int64_t dd;
        acc_sum(d.acc[t & 1], K, k, c, dd);
        L.Lc[k] = c;
        L.Ld[k] = dd;
        if (k < K) {
            L.open[k] = d.open[k];
            L.otabu[k] = d.open_tabu[k];
            L.orot[k] = 1;
        }
    }
}

// One element of a walk: the dense visit's terms while c < b2 and the base is
// a closed row of the block; the first c >= b2 ends the walk (the list is
// sorted, so no later element contributes).
#define FS_SPARSE_STEP(c, id)                                                              \
    do {                                                                                   \
        if (act && (c) < b2) {                                                             \
            const int32_t row = s_rowof[(id)];                                             \
            if (row >= 0)                                                                  \
                visit_sparse((c), b1, b2, o1, g1c, g1d, g2c, g2d, R, s_t1c + row,          \
                             s_t1d + row, L.bc + row * K, L.bd + row * K);                 \
        } else {                                                                           \
            act = false;                                                                   \
        }                                                                                  \
    } while (0)

constexpr int kSparseQ = 128;   // queued walks per wave: below 64 + 64 before a drain

// One workgroup = base block g x mission chunk sp.  Each wave takes 256
// missions at a time, four consecutive ones per lane (16-byte loads of the
// state and of each head rank, all in flight together), and walks their
// head ranks.  A mission still below b2 after the head is queued in LDS
// (ballot + mbcnt; the queue length is wave-uniform); 64 queued walks at a
// time then continue on the mission-major lists with every lane busy, each
// lane gathering its mission's state and eight ranks of its list (32
// contiguous bytes of costs, 8 of ids) in one round, and going on alone in
// the rare case that it needs more.  A wave thus waits for one round of
// loads per 256 missions plus one per 64 continued walks, instead of one
// per rank batch of every group of 64 missions.
// Packed lists: a key is below the threshold of b2 exactly when its cost is
// below b2 (sentinel keys, kNarrowTop << 6 | id, never are).
__device__ __forceinline__ uint32_t packed_threshold(int32_t b2)
{
    return b2 <= 0 ? 0u : ((uint32_t)b2 >= kNarrowTop ? kNarrowTop << 6 : (uint32_t)b2 << 6);
}

#define FS_SPARSE_KEY(key)                                                                 \
    do {                                                                                   \
        if (act && (key) < thr) {                                                          \
            const int32_t row = s_rowof[(key) & 63];                                       \
            if (row >= 0)                                                                  \
                visit_sparse((int32_t)((key) >> 6), b1, b2, o1, g1c, g1d, g2c, g2d, R,     \
                             s_t1c + row, s_t1d + row, L.bc + row * K, L.bd + row * K);    \
        } else {                                                                           \
            act = false;                                                                   \
        }                                                                                  \
    } while (0)

template <int BS, bool PACKED>
__global__ __launch_bounds__(BS, 8) void k_sweep_sparse(const InstDesc *__restrict__ descs,
                                                     const Tile *__restrict__ tiles, int32_t step)
{
    const Tile tl = sweep_tile(descs, tiles);
    const InstDesc &d = descs[tl.inst];
    if (!d.active) return;
    const int32_t t = step - d.start_step;
    if (t < 1 || t > d.N) return;
    // (the state, the block's rows and the slot inputs are loaded where they
    // are used: measured faster here than one round waited for by every wave)
    const SolveState st = *d.st;
    const bool scoring = d.nsplit == 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t K = d.K, R = d.R;
    const SweepLds L = carve_lds(smem, kSparseW, K);
    __shared__ int32_t s_jrow[kSparseW], s_jslot[kSparseW], s_jtabu[kSparseW],
        s_jhel[kSparseW], s_rowof[kSparseW];
    __shared__ int32_t s_t1c[kSparseW];
    __shared__ u64 s_t1d[kSparseW];
    __shared__ int32_t s_nrows;
    __shared__ Candidate s_red[BS / 64 + 1];
    __shared__ int32_t s_q[BS / 64][kSparseQ];

    if (threadIdx.x < kSparseW) {
        s_t1c[threadIdx.x] = 0;
        s_t1d[threadIdx.x] = 0;
        SparseSetup su;
        const int32_t b = tl.g * kSparseW + (int32_t)threadIdx.x;
        su.inb = b < d.B;
        su.slot = su.inb ? gptr(d.base_slot)[b] : -1;
        su.tabu = su.inb ? gptr(d.base_tabu)[b] : 0;
        sparse_rows(su, tl.g, s_jrow, s_jslot, s_jtabu, s_jhel, s_rowof, &s_nrows);
    }
    if (scoring) load_slot_inputs(d, t, L, false);
    if (st.stopped) return;
    if (tl.g == 0 && tl.sp == 0) sweep_housekeeping(d, t);
    for (int q = threadIdx.x; q < kSparseW * K; q += BS) {
        L.bd[q] = 0;
        L.bc[q] = 0;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t m0 = tl.sp * d.chunk, m1 = min(d.Mp, m0 + d.chunk);
    const int64_t Mp = d.Mp;
    typedef const __attribute__((address_space(1))) uint32_t gu32;
    typedef const __attribute__((address_space(1))) uint64_t gu64;
    const int32_t *hc = d.lst_cost + (int64_t)tl.g * kSparseHead * Mp;
    const unsigned char *hi = d.lst_id + (int64_t)tl.g * kSparseHead * Mp;
    const int32_t *tc = d.mm_cost + (int64_t)tl.g * Mp * kSparseW;
    const unsigned char *ti = d.mm_id + (int64_t)tl.g * Mp * kSparseW;
    int32_t *myq = s_q[wave];
    int32_t qlen = 0;

    // The continued walks of queue entries [0, n): one per lane, ranks from
    // kSparseHead on.
    auto drain = [&](int32_t n) {
        __builtin_amdgcn_wave_barrier();
        const bool have = lane < n;
        const int32_t m = have ? myq[lane] : m0;
        const gv4i *myc = (const gv4i *)(tc + (int64_t)m * kSparseW);
        const gu64 *myi = (const gu64 *)(ti + (int64_t)m * kSparseW);
        // the state and the first eight ranks go out together
        const int32_t b1 = ((const gi32 *)d.b1)[m], b2 = ((const gi32 *)d.b2)[m],
                      o1 = ((const gi32 *)d.o1)[m];
        v4i c0 = myc[0], c1 = myc[1];
        uint64_t ids = PACKED ? 0 : myi[0];
        const int32_t g1c = b1 <= R, g1d = g1c ? b1 : 0;
        const int32_t g2c = b2 <= R, g2d = g2c ? b2 : 0;
        const uint32_t thr = packed_threshold(b2);
        bool act = have;
        for (int32_t r8 = 0; r8 < kSparseW / 8; ++r8) {
            if (r8 > 0) {
                if (__builtin_amdgcn_ballot_w64(act) == 0) break;
                if (act) {
                    c0 = myc[2 * r8];
                    c1 = myc[2 * r8 + 1];
                    if (!PACKED) ids = myi[r8];
                }
            }
            int32_t cs[8];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                cs[e] = c0[e];
                cs[4 + e] = c1[e];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                if (r8 == 0 && e < kSparseHead) continue;
                if (PACKED) {
                    FS_SPARSE_KEY((uint32_t)cs[e]);
                } else {
                    FS_SPARSE_STEP(cs[e], (int32_t)((ids >> (8 * e)) & 0xFF));
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    };

    for (int32_t mw = m0 + wave * 256; mw < m1; mw += BS * 4) {
        const int32_t mq = mw + 4 * lane;    // this lane's four missions mq .. mq + 3
        const bool in = mq < m1;             // (Mp and the chunk are multiples of 4)
        const int32_t mc = in ? mq : m0;     // in-bounds address for idle lanes
        v4i hcs[kSparseHead];
        uint32_t hid[kSparseHead];
#pragma unroll
        for (int r = 0; r < kSparseHead; ++r) {
            hcs[r] = *(const gv4i *)(hc + r * Mp + mc);
            hid[r] = PACKED ? 0u : *(const gu32 *)(hi + r * Mp + mc);
        }
        const v4i vb1 = *(const gv4i *)(d.b1 + mc), vb2 = *(const gv4i *)(d.b2 + mc),
                  vo1 = *(const gv4i *)(d.o1 + mc);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int32_t b1 = vb1[e], b2 = in ? vb2[e] : INT32_MIN, o1 = vo1[e];
            const int32_t g1c = b1 <= R, g1d = g1c ? b1 : 0;
            const int32_t g2c = b2 <= R, g2d = g2c ? b2 : 0;
            const uint32_t thr = packed_threshold(b2);
            bool act = in;
#pragma unroll
            for (int r = 0; r < kSparseHead; ++r) {
                if (PACKED) {
                    FS_SPARSE_KEY((uint32_t)hcs[r][e]);
                } else {
                    FS_SPARSE_STEP(hcs[r][e], (int32_t)((hid[r] >> (8 * e)) & 0xFF));
                }
            }
            // walks that go on past the head join the queue
            const u64 mask = __builtin_amdgcn_ballot_w64(act);
            if (mask == 0) continue;
            if (act) {
                const int32_t at = (int32_t)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask,
                                                                     (uint32_t)qlen));
                myq[at] = mq + e;
            }
            qlen = __builtin_amdgcn_readfirstlane(qlen + (int32_t)__builtin_popcountll(mask));
            if (qlen >= 64) {
                drain(64);
                qlen -= 64;
                const int32_t rest = lane < qlen ? myq[64 + lane] : 0;
                __builtin_amdgcn_wave_barrier();
                if (lane < qlen) myq[lane] = rest;
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    if (qlen > 0) drain(qlen);
    __syncthreads();
    const int32_t nrows = s_nrows;
    if (scoring) {
        __shared__ int64_t s_t1ds[kSparseW];
        if (threadIdx.x < kSparseW) s_t1ds[threadIdx.x] = (int64_t)s_t1d[threadIdx.x];
        __syncthreads();
        score_group<BS>(d, st, nrows, 1, t, tl.g, s_jrow, s_jtabu, s_jhel, L, s_t1c, s_t1ds,
                            s_red, s_jslot);
    } else {
        // this chunk's [T1, bin_0 .. bin_{K-1}] per row, added into the
        // block's sums (nonzero entries only; integer atomics, exact in any
        // order); k_score_sparse scores the block after every chunk
        const int32_t K1 = K + 1;
        const int64_t base = (int64_t)tl.g * kSparseW * K1;
        unsigned int *pc = reinterpret_cast<unsigned int *>(d.part_cov) + base;
        u64 *pd = reinterpret_cast<u64 *>(d.part_dist) + base;
        for (int32_t idx = threadIdx.x; idx < nrows * K1; idx += BS) {
            const int32_t r = idx / K1, k = idx - r * K1;
            const int32_t c = k == 0 ? s_t1c[r] : L.bc[r * K + k - 1];
            const u64 dd = k == 0 ? s_t1d[r] : L.bd[r * K + k - 1];
            if (c) gatomic_add(pc + idx, (unsigned int)c);
            if (dd) gatomic_add(pd + idx, dd);
        }
    }
}

#undef FS_SPARSE_STEP
#undef FS_SPARSE_KEY

// Scores a quarter of one base block (16 of its closed rows, kScoreParts
// workgroups per block) from the block's sums over the mission chunks (added
// by the sweep's chunks) and clears them for the next iteration (all 16 row
// slots: the next iteration's rows may differ).  Candidate kScoreParts * g + part.
// (score_part: the work of one scoring workgroup; signal: the refresh
// workgroups of the same launch wait for it, see refresh_tile.)
template <int BS>
__device__ __forceinline__ void score_part(const InstDesc *__restrict__ descs, const Tile tl,
                                           int32_t step, bool signal);

template <int BS>
__global__ __launch_bounds__(BS) void k_score_sparse(const InstDesc *__restrict__ descs,
                                                     const Tile *__restrict__ tiles, int32_t step)
{
    const Tile tl = tiles ? tiles[blockIdx.x]
                          : Tile{0, (int32_t)blockIdx.x / kScoreParts,
                                 (int32_t)blockIdx.x % kScoreParts, 0};
    score_part<BS>(descs, tl, step, false);
}

template <int BS>
__device__ __forceinline__ void score_part(const InstDesc *__restrict__ descs, const Tile tl,
                                           int32_t step, bool signal)
{
    const InstDesc &d = descs[tl.inst];
    if (!d.active) return;
    const int32_t t = step - d.start_step;
    if (t < 1 || t > d.N) return;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int RP = kSparseW / kScoreParts;   // rows per part
    const int32_t K = d.K, K1 = K + 1, part = tl.sp, r0 = part * RP;
    const SweepLds L = carve_lds(smem, RP, K);
    __shared__ int32_t s_jrow[kSparseW], s_jslot[kSparseW], s_jtabu[kSparseW],
        s_jhel[kSparseW], s_rowof[kSparseW];
    __shared__ int32_t s_t1c[RP];
    __shared__ int64_t s_t1d[RP];
    __shared__ int32_t s_nrows;
    __shared__ Candidate s_red[BS / 64 + 1];
    // this part's sums go out with the row and slot loads and are waited for
    // once
    constexpr int PER = (RP * (kSparseMaxK + 1) + BS - 1) / BS;
    const int64_t base = ((int64_t)tl.g * kSparseW + r0) * K1;
    int32_t pcv[PER];
    int64_t pdv[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int32_t idx = threadIdx.x + i * BS;
        const int32_t at = idx < RP * K1 ? idx : 0;   // (in bounds: loaded, then dropped)
        pcv[i] = gptr(d.part_cov)[base + at];
        pdv[i] = gptr(d.part_dist)[base + at];
    }
    const SparseSetup su = sparse_setup(d, t, tl.g);
#pragma unroll
    for (int i = 0; i < PER; ++i) asm volatile("" ::"v"(pcv[i]), "v"(pdv[i]));
    const SolveState &st = su.st;
    if (st.stopped) return;
    if (threadIdx.x < kSparseW)
        sparse_rows(su, tl.g, s_jrow, s_jslot, s_jtabu, s_jhel, s_rowof, &s_nrows);
    sparse_slot_inputs(d, t, su, L);
    __syncthreads();
    const int32_t nr = min(max(s_nrows - r0, 0), RP);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int32_t idx = threadIdx.x + i * BS;
        if (idx >= RP * K1) continue;
        const int32_t c = pcv[i];
        const int64_t dd = pdv[i];
        gptr(d.part_cov)[base + idx] = 0;
        gptr(d.part_dist)[base + idx] = 0;
        if (idx >= nr * K1) continue;
        const int32_t r = idx / K1, k = idx - r * K1;
        if (k == 0) {
            s_t1c[r] = c;
            s_t1d[r] = dd;
        } else {
            L.bc[r * K + k - 1] = c;
            L.bd[r * K + k - 1] = (u64)dd;
        }
    }
    __syncthreads();
    score_group<BS>(d, st, nr, 1, t, kScoreParts * tl.g + part, s_jrow + r0, s_jtabu + r0,
                    s_jhel + r0, L, s_t1c, s_t1d, s_red, s_jslot + r0);
    // (thread 0 wrote the candidate; its release publishes it)
    if (signal && threadIdx.x == 0)
        __hip_atomic_fetch_add(&d.st->score_done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The block scores and the refresh of one iteration of the sparse sweep in
// one launch (one instance): workgroups [0, nscore) score base-block parts and
// never wait; the others are refresh workgroups, which wait for every
// scoring workgroup's candidate (they are dispatched after them, so the wait
// always ends) and then refresh as usual.  Saves a launch per iteration and
// overlaps the refresh workgroups' start with the scoring.
template <int MPT, bool TY, int BS>
__global__ __launch_bounds__(BS) void k_score_refresh(const InstDesc *__restrict__ descs,
                                                      int32_t nscore, int32_t step)
{
    const int32_t b = (int32_t)blockIdx.x;
    if (b < nscore)
        score_part<BS>(descs, Tile{0, b / kScoreParts, b % kScoreParts, 0}, step, true);
    else
        refresh_tile<MPT, TY, BS>(descs, Tile{0, b - nscore, 0, 0}, step, b - nscore, true);
}

// Sums the chunk partials of one row group of a split instance and scores it.
template <int J>
__global__ __launch_bounds__(kBlock) void k_score(const InstDesc *__restrict__ descs,
                                                  const Tile *__restrict__ tiles, int32_t step)
{
    const Tile tl = group_tile(tiles);
    const InstDesc &d = descs[tl.inst];
    if (!d.active) return;
    const int32_t t = step - d.start_step;
    if (t < 1 || t > d.N) return;
    const SolveState st = *d.st;
    if (st.stopped) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t K = d.K, K2 = K + 2;
    const SweepLds L = carve_lds(smem, J, K);
    __shared__ int32_t s_jrow[J], s_jtabu[J], s_jhel[J];
    __shared__ int32_t s_sum_c[2 * J];
    __shared__ int64_t s_sum_d[2 * J];
    __shared__ Candidate s_red[kBlock / 64 + 1];
    const int32_t nclosed = d.nclosed;
    if (threadIdx.x < J) {
        const int32_t js = tl.g * J + threadIdx.x;
        const int32_t jc = js < nclosed ? js : 0;
        s_jrow[threadIdx.x] = d.closed[jc];
        s_jtabu[threadIdx.x] = d.closed_tabu[jc];
        s_jhel[threadIdx.x] = d.typed ? d.closed_hel[jc] : 0;
    }
    load_slot_inputs(d, t, L, d.typed != 0);
    for (int32_t idx = threadIdx.x; idx < J * K2; idx += kBlock) {
        const int32_t r = idx / K2, k = idx - r * K2;
        const int32_t js = tl.g * J + r;
        int32_t c = 0;
        int64_t dd = 0;
        if (js < nclosed) {
            for (int32_t sp = 0; sp < d.nsplit; ++sp) {
                const int64_t at = ((int64_t)sp * nclosed + js) * K2 + k;
                c += d.part_cov[at];
                dd += d.part_dist[at];
            }
        }
        if (k < 2) {
            s_sum_c[2 * r + k] = c;
            s_sum_d[2 * r + k] = dd;
        } else {
            L.bc[r * K + k - 2] = c;
            L.bd[r * K + k - 2] = (u64)dd;
        }
    }
    __syncthreads();
    score_group<kBlock>(d, st, J, 2, t, tl.g, s_jrow, s_jtabu, s_jhel, L, s_sum_c, s_sum_d, s_red);
}

// ---------------------------------------------------------------- outputs

// One workgroup per instance: best placement in ascending id order, score,
// and the first iteration whose refreshed value disagreed with its score.
__global__ __launch_bounds__(kBlock) void k_outputs(const InstDesc *__restrict__ descs,
                                                    fs_score *__restrict__ scores,
                                                    int32_t *__restrict__ errors)
{
    const InstDesc &d = descs[blockIdx.x];
    if (!d.active) return;
    const int32_t K = d.K;
    for (int32_t k = threadIdx.x; k < K; k += kBlock) {
        const int32_t v = d.best_open[k];
        int32_t pos = 0;
        for (int32_t q = 0; q < K; ++q) pos += d.best_open[q] < v;
        d.best_sorted[pos] = v;
        d.best_rot_sorted[pos] = d.open_rot[k];   // a slot keeps its vehicle
        if (d.best_out) d.best_out[pos] = v;
        if (d.best_rot_out) d.best_rot_out[pos] = d.open_rot[k];
    }
    if (threadIdx.x == 0) {
        const SolveState *st = d.st;
        fs_score sc;
        sc.coverage = st->best_cov;
        sc.best_iter = st->best_iter;
        sc.distance = st->best_dist;
        scores[blockIdx.x] = sc;
        int32_t err = st->error ? st->err_iter : 0;
        // the state after the last move was refreshed too: check it
        if (!err && d.N >= 1 && !st->stopped) {
            int32_t gc;
            int64_t gd;
            acc_sum(d.acc[(d.N + 1) & 1], K, 0, gc, gd);
            if (gc != st->cur_cov || gd != st->cur_dist) err = d.N + 1;
        }
        errors[blockIdx.x] = err;
    }
}

// Nearest open base of each mission of the best placement (ascending ids, so
// the first strict minimum is the lowest id among equal costs), or -1 beyond
// R.  Tiles of 64 missions (the refresh tiles); one mission per thread of the
// first wave.
template <int MPT>
__global__ __launch_bounds__(kBlock) void k_assign(const InstDesc *__restrict__ descs,
                                                   const Tile *__restrict__ tiles)
{
    const Tile tl = tiles[blockIdx.x];
    const InstDesc &d = descs[tl.inst];
    if (!d.active || !d.assign_out) return;
    if (threadIdx.x >= MPT) return;
    const int32_t m = tl.g * MPT + threadIdx.x;
    if (m >= d.M) return;
    int32_t v = INT32_MAX, who = -1;
    const bool rot_only = d.rho && d.rho[m] != 0;
    for (int32_t k = 0; k < d.K; ++k) {
        if (rot_only && !d.best_rot_sorted[k]) continue;
        const int32_t id = d.best_sorted[k];
        const int32_t c = d.C[(int64_t)id * d.ldc + m];
        if (c < v) {
            v = c;
            who = id;
        }
    }
    d.assign_out[m] = v <= d.R ? who : -1;
}

// ---------------------------------------------------------------- persistent search (A6)
//
// One workgroup runs one instance's whole search: every iteration's sweep,
// argmax, move and state refresh, with the per-mission state (b1, b2, o1),
// the open and closed lists with their tabu expiries, and G / L_k resident in
// LDS.  Workgroups never wait for one another, so a ragged batch of instances
// is a single launch of the whole iteration loop (after the base ranking and
// the initial state), and a small instance pays no launch per iteration.
// The arithmetic is the multi-workgroup engine's: the same terms per element
// (visit_hit), the same move order and admissibility, the same commit, so
// the trajectory is identical.
//
// Sweep: each wave takes kSoloJ closed rows at a time and streams every
// mission of them (16-byte row loads, b2 from LDS); elements below b2 are
// queued per wave and scored 64 at a time into the wave's own bins; the wave
// then scores its kSoloJ x K moves and keeps its best candidate.  Refresh:
// one mission per thread over the K open rows (sixteen loads in flight).

constexpr int kSoloWaves = 8;
constexpr int kSoloBlock = 64 * kSoloWaves;
constexpr int kSoloJ = 4;
constexpr int kSoloU = 2;
constexpr int kSoloQ = 128;

struct SoloLayout {
    uint32_t Ld, nLd, bd, b1, b2, Lc, nLc, bc, open, otabu, closed, ctabu, qc, qm, o1, tab, total;
};

// tab_B > 0: the instance's B x Mp cost table is staged in LDS as well (row
// pitch Mp), so that the loop touches no global memory but its trace.
__host__ __device__ inline SoloLayout solo_layout(int32_t Mp, int32_t K, int32_t ncl,
                                                  int32_t tab_B = 0)
{
    SoloLayout L{};
    uint32_t o = 0;
    auto take = [&o](uint32_t bytes) {
        const uint32_t r = o;
        o += (bytes + 15u) & ~15u;
        return r;
    };
    const uint32_t bins = (uint32_t)(kSoloWaves * kSoloJ * K);
    L.Ld = take(8u * (uint32_t)(K + 1));
    L.nLd = take(8u * (uint32_t)(K + 1));
    L.bd = take(8u * bins);
    L.b1 = take(4u * (uint32_t)Mp);
    L.b2 = take(4u * (uint32_t)Mp);
    L.Lc = take(4u * (uint32_t)(K + 1));
    L.nLc = take(4u * (uint32_t)(K + 1));
    L.bc = take(4u * bins);
    L.open = take(4u * (uint32_t)K);
    L.otabu = take(4u * (uint32_t)K);
    L.closed = take(4u * (uint32_t)ncl);
    L.ctabu = take(4u * (uint32_t)ncl);
    L.qc = take(4u * kSoloWaves * kSoloQ);
    L.qm = take(4u * kSoloWaves * kSoloQ);
    L.o1 = take((uint32_t)Mp);
    L.tab = take(4u * (uint32_t)tab_B * (uint32_t)Mp);
    L.total = o;
    return L;
}

template <bool TAB>
__global__ __launch_bounds__(kSoloBlock) void k_solo(const InstDesc *__restrict__ descs,
                                                     const Tile *__restrict__ order)
{
    const InstDesc &d = descs[order[blockIdx.x].inst];
    if (!d.active || d.N < 1) return;
    const int32_t K = d.K, M = d.M, Mp = d.Mp, R = d.R, N = d.N, T = d.T, mode = d.mode;
    const int32_t nclosed = d.nclosed, ncl = max(nclosed, 1);
    const int lane = threadIdx.x & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    extern __shared__ __align__(16) unsigned char smem[];
    const SoloLayout LO = solo_layout(Mp, K, ncl, TAB ? d.B : 0);
    // the cost table: device memory, or its LDS copy (row pitch Mp)
    int32_t *s_tab = reinterpret_cast<int32_t *>(smem + LO.tab);
    const int32_t *Ctab = TAB ? s_tab : d.C;
    const int64_t ldc = TAB ? (int64_t)Mp : d.ldc;
    u64 *s_Ld = reinterpret_cast<u64 *>(smem + LO.Ld);
    u64 *s_nLd = reinterpret_cast<u64 *>(smem + LO.nLd);
    int32_t *s_b1 = reinterpret_cast<int32_t *>(smem + LO.b1);
    int32_t *s_b2 = reinterpret_cast<int32_t *>(smem + LO.b2);
    int32_t *s_Lc = reinterpret_cast<int32_t *>(smem + LO.Lc);
    int32_t *s_nLc = reinterpret_cast<int32_t *>(smem + LO.nLc);
    int32_t *s_open = reinterpret_cast<int32_t *>(smem + LO.open);
    int32_t *s_otabu = reinterpret_cast<int32_t *>(smem + LO.otabu);
    int32_t *s_closed = reinterpret_cast<int32_t *>(smem + LO.closed);
    int32_t *s_ctabu = reinterpret_cast<int32_t *>(smem + LO.ctabu);
    unsigned char *s_o1 = smem + LO.o1;
    // this wave's bins and hit queue
    int32_t *bc = reinterpret_cast<int32_t *>(smem + LO.bc) + wave * kSoloJ * K;
    u64 *bd = reinterpret_cast<u64 *>(smem + LO.bd) + wave * kSoloJ * K;
    int32_t *qc = reinterpret_cast<int32_t *>(smem + LO.qc) + wave * kSoloQ;
    int32_t *qm = reinterpret_cast<int32_t *>(smem + LO.qm) + wave * kSoloQ;
    __shared__ Candidate s_red[kSoloWaves];
    __shared__ SolveState s_st;
    __shared__ int32_t s_valid, s_improved;

    // the state of S_1 (engine_init), the lists and their expiries
    for (int32_t m = threadIdx.x; m < Mp; m += kSoloBlock) {
        s_b1[m] = d.b1[m];
        s_b2[m] = d.b2[m];
        s_o1[m] = (unsigned char)(d.o1[m] & 0xFF);
    }
    for (int32_t k = threadIdx.x; k < K; k += kSoloBlock) {
        s_open[k] = d.open[k];
        s_otabu[k] = d.open_tabu[k];
    }
    for (int32_t js = threadIdx.x; js < ncl; js += kSoloBlock) {
        s_closed[js] = d.closed[js];
        s_ctabu[js] = d.closed_tabu[js];
    }
    for (int32_t k = threadIdx.x; k <= K; k += kSoloBlock) {
        int32_t c;
        int64_t dd;
        acc_sum(d.acc[1], K, k, c, dd);
        s_Lc[k] = c;
        s_Ld[k] = (u64)dd;
    }
    if (TAB) {
        // (padding columns M .. Mp-1 are never compared: their b2 is INT32_MIN)
        const int32_t B = d.B, nq4 = Mp >> 2;
        for (int32_t e = threadIdx.x; e < B * nq4; e += kSoloBlock) {
            const int32_t b = e / nq4, q = e - b * nq4;
            v4i v;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int32_t m = 4 * q + i;
                v[i] = m < M ? d.C[(int64_t)b * d.ldc + m] : INT32_MAX;
            }
            *reinterpret_cast<v4i *>(s_tab + (int64_t)b * Mp + 4 * q) = v;
        }
    }
    if (threadIdx.x == 0) s_st = *d.st;
    __syncthreads();

    const int32_t nq = Mp >> 2;
    const int32_t ngroups = nclosed > 0 ? (nclosed + kSoloJ - 1) / kSoloJ : 0;
    for (int32_t t = 1; t <= N; ++t) {
        if (s_st.stopped) {
            // local search ended earlier: the iteration makes no move
            if (threadIdx.x == 0) write_record(d, t, s_st, 0, -1, -1);
            continue;
        }
        const int32_t Gc = s_Lc[0];
        const int64_t Gd = (int64_t)s_Ld[0];
        const int32_t cur_c = s_st.cur_cov, best_c = s_st.best_cov;
        const int64_t cur_d = s_st.cur_dist, best_d = s_st.best_dist;
        Candidate mine = no_cand();

        // ---- sweep: kSoloJ closed rows per wave at a time
        for (int32_t g = wave; g < ngroups; g += kSoloWaves) {
            int32_t js[kSoloJ], jr[kSoloJ];
            bool rv[kSoloJ];
            const v4i *rows[kSoloJ];
#pragma unroll
            for (int r = 0; r < kSoloJ; ++r) {
                js[r] = g * kSoloJ + r;
                rv[r] = js[r] < nclosed;
                jr[r] = s_closed[rv[r] ? js[r] : 0];
                rows[r] = reinterpret_cast<const v4i *>(Ctab + (int64_t)jr[r] * ldc);
            }
            for (int32_t idx = lane; idx < kSoloJ * K; idx += 64) {
                bc[idx] = 0;
                bd[idx] = 0;
            }
            int32_t t1c[kSoloJ];
            int64_t t1d[kSoloJ];
#pragma unroll
            for (int r = 0; r < kSoloJ; ++r) {
                t1c[r] = 0;
                t1d[r] = 0;
            }
            int32_t qlen = 0;
            // score queue entries [0, n), one per lane (a macro: the per-row
            // sums stay in registers)
#define FS_SOLO_DRAIN(n)                                                                   \
    do {                                                                                   \
        __builtin_amdgcn_wave_barrier();                                                   \
        if (lane < (n)) {                                                                  \
            const int32_t c_ = qc[lane], mr_ = qm[lane];                                   \
            const int32_t m_ = mr_ & 0xFFFFFF, r_ = mr_ >> 24;                             \
            const int32_t b1_ = s_b1[m_], b2_ = s_b2[m_], o1_ = s_o1[m_];                  \
            const int32_t g1c_ = b1_ <= R, g1d_ = g1c_ ? b1_ : 0;                          \
            const int32_t g2c_ = b2_ <= R, g2d_ = g2c_ ? b2_ : 0;                          \
            const int32_t v1_ = min(c_, b1_), u_ = max(c_, b1_);                           \
            const int32_t cv_ = v1_ <= R;                                                  \
            const int32_t tc_ = cv_ - g1c_, td_ = (cv_ ? v1_ : 0) - g1d_;                  \
            _Pragma("unroll") for (int q_ = 0; q_ < kSoloJ; ++q_)                          \
            {                                                                              \
                t1c[q_] += r_ == q_ ? tc_ : 0;                                             \
                t1d[q_] += r_ == q_ ? (int64_t)td_ : 0;                                    \
            }                                                                              \
            const int32_t cu_ = u_ <= R;                                                   \
            const int32_t dc_ = cu_ - g2c_, dd_ = (cu_ ? u_ : 0) - g2d_;                   \
            if (dc_ | dd_) {                                                               \
                atomicAdd(bc + r_ * K + o1_, dc_);                                         \
                atomicAdd(bd + r_ * K + o1_, (u64)(int64_t)dd_);                           \
            }                                                                              \
        }                                                                                  \
        __builtin_amdgcn_wave_barrier();                                                   \
    } while (0)
            for (int32_t q0 = 0; q0 < nq; q0 += 64 * kSoloU) {
                v4i cv[kSoloU][kSoloJ], vb2[kSoloU];
#pragma unroll
                for (int u = 0; u < kSoloU; ++u) {
                    const int32_t q = min(q0 + u * 64 + lane, nq - 1);
#pragma unroll
                    for (int r = 0; r < kSoloJ; ++r)
                        cv[u][r] = TAB ? rows[r][q]
                                       : *(const __attribute__((address_space(1))) v4i *)(rows[r] + q);
                    vb2[u] = *reinterpret_cast<const v4i *>(s_b2 + 4 * q);
                }
#pragma unroll
                for (int u = 0; u < kSoloU; ++u) {
                    const int32_t q = q0 + u * 64 + lane;
                    if (q >= nq) vb2[u] = (v4i)(INT32_MIN);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
#pragma unroll
                        for (int r = 0; r < kSoloJ; ++r) {
                            const bool hit = rv[r] && cv[u][r][e] < vb2[u][e];
                            const u64 mask = __builtin_amdgcn_ballot_w64(hit);
                            if (mask == 0) continue;
                            if (hit) {
                                const int32_t at = (int32_t)__builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(mask >> 32),
                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, (uint32_t)qlen));
                                qc[at] = cv[u][r][e];
                                qm[at] = (4 * q + e) | (r << 24);
                            }
                            qlen = __builtin_amdgcn_readfirstlane(
                                qlen + (int32_t)__builtin_popcountll(mask));
                            if (qlen >= 64) {
                                FS_SOLO_DRAIN(64);
                                qlen -= 64;
                                int32_t c2 = 0, m2 = 0;
                                if (lane < qlen) {
                                    c2 = qc[64 + lane];
                                    m2 = qm[64 + lane];
                                }
                                __builtin_amdgcn_wave_barrier();
                                if (lane < qlen) {
                                    qc[lane] = c2;
                                    qm[lane] = m2;
                                }
                                __builtin_amdgcn_wave_barrier();
                            }
                        }
                    }
                }
            }
            if (qlen > 0) FS_SOLO_DRAIN(qlen);
#undef FS_SOLO_DRAIN
            __builtin_amdgcn_wave_barrier();
            // the rows' common terms, then this group's moves
#pragma unroll
            for (int r = 0; r < kSoloJ; ++r) {
                t1c[r] = wave_sum_i32(t1c[r]);
                t1d[r] = wave_sum_i64(t1d[r]);
            }
#pragma unroll
            for (int r = 0; r < kSoloJ; ++r) {
                if (!rv[r]) continue;
                for (int32_t k = lane; k < K; k += 64) {
                    const int32_t idx = r * K + k;
                    const int32_t cov = Gc + s_Lc[1 + k] + t1c[r] + bc[idx];
                    const int64_t dist = Gd + (int64_t)s_Ld[1 + k] + t1d[r] + (int64_t)bd[idx];
                    const bool adm = mode == 1 ? better(cov, dist, cur_c, cur_d)
                                               : (s_otabu[k] < t && s_ctabu[js[r]] < t) ||
                                                     better(cov, dist, best_c, best_d);
                    if (adm) {
                        Candidate c;
                        c.cov = cov;
                        c.dist = dist;
                        c.i_base = s_open[k];
                        c.j_base = jr[r];
                        c.slots = (uint32_t)k | ((uint32_t)js[r] << kSlotBits);
                        c.key = 0;
                        if (cand_better<false>(c, mine)) mine = c;
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        mine = wave_best<false>(mine);
        if (lane == 0) s_red[wave] = mine;
        __syncthreads();

        // ---- argmax and commit (the multi-workgroup refresh's leader)
        if (threadIdx.x == 0) {
            Candidate best = s_red[0];
            for (int w = 1; w < kSoloWaves; ++w)
                if (cand_better<false>(s_red[w], best)) best = s_red[w];
            SolveState s = s_st;
            const bool valid = cand_valid(best);
            int32_t improved = 0;
            if (!valid && mode == 1) {
                s.stopped = 1;   // local optimum: the placement stays as it is
                write_record(d, t, s, 0, -1, -1);
            } else {
                if (valid) {
                    s.cur_cov = best.cov;
                    s.cur_dist = best.dist;
                    if (better(best.cov, best.dist, s.best_cov, s.best_dist)) {
                        s.best_cov = best.cov;
                        s.best_dist = best.dist;
                        s.best_iter = t;
                        improved = 1;
                    }
                    s.have_last = 1;
                    s.last_key = best.key;
                    const int32_t i_slot = cand_i_slot(best), j_slot = cand_j_slot(best);
                    s_open[i_slot] = best.j_base;
                    s_otabu[i_slot] = t + T;
                    s_closed[j_slot] = best.i_base;
                    s_ctabu[j_slot] = t + T;
                }
                write_record(d, t, s, valid, best.i_base, best.j_base);
            }
            s_st = s;
            s_valid = valid;
            s_improved = improved;
        }
        for (int32_t k = threadIdx.x; k <= K; k += kSoloBlock) {
            s_nLc[k] = 0;
            s_nLd[k] = 0;
        }
        __syncthreads();
        if (!s_valid) continue;   // no move: the placement and its state are unchanged
        if (s_improved)
            for (int32_t k = threadIdx.x; k < K; k += kSoloBlock) d.best_open[k] = s_open[k];

        // ---- state of the new placement
        int32_t gc = 0;
        int64_t gd = 0;
        for (int32_t m = threadIdx.x; m < M; m += kSoloBlock) {
            const int32_t *col = Ctab + m;
            int32_t v1 = INT32_MAX, i1 = INT32_MAX, s1 = 0, v2 = INT32_MAX;
            constexpr int UNR = 16;
            for (int32_t k0 = 0; k0 < K; k0 += UNR) {
                int32_t c[UNR], id[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int32_t k = k0 + u;
                    id[u] = k < K ? s_open[k] : 0;
                    c[u] = k < K ? col[(int64_t)id[u] * ldc] : INT32_MAX;
                }
#pragma unroll
                for (int u = 0; u < UNR; ++u) {
                    const int32_t k = k0 + u;
                    if (k < K) {
                        if (c[u] < v1 || (c[u] == v1 && id[u] < i1)) {
                            v2 = v1;
                            v1 = c[u];
                            i1 = id[u];
                            s1 = k;
                        } else if (c[u] < v2) {
                            v2 = c[u];
                        }
                    }
                }
            }
            s_b1[m] = v1;
            s_b2[m] = v2;
            s_o1[m] = (unsigned char)s1;
            const int32_t g1c = v1 <= R, g1d = g1c ? v1 : 0;
            const int32_t g2c = v2 <= R, g2d = g2c ? v2 : 0;
            const int32_t dc = g2c - g1c, dd = g2d - g1d;
            if (dc | dd) {
                atomicAdd(&s_nLc[1 + s1], dc);
                atomicAdd(&s_nLd[1 + s1], (u64)(int64_t)dd);
            }
            gc += g1c;
            gd += g1d;
        }
        gc = wave_sum_i32(gc);
        gd = wave_sum_i64(gd);
        if (lane == 0) {
            atomicAdd(&s_nLc[0], gc);
            atomicAdd(&s_nLd[0], (u64)gd);
        }
        __syncthreads();
        // the recounted value must be the chosen move's score
        if (threadIdx.x == 0 && (s_nLc[0] != s_st.cur_cov || (int64_t)s_nLd[0] != s_st.cur_dist) &&
            !s_st.error) {
            s_st.error = 1;
            s_st.err_iter = t + 1;
        }
        for (int32_t k = threadIdx.x; k <= K; k += kSoloBlock) {
            s_Lc[k] = s_nLc[k];
            s_Ld[k] = s_nLd[k];
        }
        __syncthreads();
    }

    // back to device memory: what the outputs read (search state, best
    // placement) and the final placement's lists and value
    for (int32_t k = threadIdx.x; k < K; k += kSoloBlock) {
        d.open[k] = s_open[k];
        d.open_tabu[k] = s_otabu[k];
    }
    for (int32_t js = threadIdx.x; js < ncl; js += kSoloBlock) {
        d.closed[js] = s_closed[js];
        d.closed_tabu[js] = s_ctabu[js];
    }
    Acc *fin = d.acc[(N + 1) & 1];
    for (int32_t q = threadIdx.x; q < kStripes * (K + 1); q += kSoloBlock) {
        const bool s0 = q < K + 1;
        fin[q].cov = s0 ? (u64)(int64_t)s_Lc[q] : 0;
        fin[q].dist = s0 ? s_Ld[q] : 0;
    }
    if (threadIdx.x == 0) *d.st = s_st;
}

// ---------------------------------------------------------------- dispatch

// A launch that carries the timing events when there are any (the dispatch
// stamps them) and is a plain launch otherwise.
template <typename... Params, typename... Args>
void launch_timed(void (*kernel)(Params...), dim3 grid, dim3 block, uint32_t lds, hipStream_t s,
                  hipEvent_t start, hipEvent_t stop, Args... args)
{
    if (start || stop)
        hipExtLaunchKernelGGL(kernel, grid, block, lds, s, start, stop, 0u, args...);
    else
        kernel<<<grid, block, lds, s>>>(args...);
}


template <int J, int U, bool VEC4, bool NT, bool Q, int NC>
fs_status launch_sweep_t(const EngineTables &t, const EngineConfig &c, int32_t step, hipStream_t s,
                         TimedLaunch &tm)
{
    if (c.typed != (NC == 2))
        return fail(FS_E_INTERNAL, "sweep kernel with %d common-term classes for a %s launch set",
                    NC, c.typed ? "typed" : "homogeneous");
    const uint32_t lds = (uint32_t)sweep_lds_bytes(J, c.Kmax);
    const bool score = t.nscore > 0;
    if (t.nsweep > 0) {
        bool launched = false;
        // 1024-thread workgroups: up to 2 rows with any variant; more rows
        // only with in-place scoring and one load in flight (LDS queues and
        // registers grow with the rows)
        if constexpr (J <= 2 || (!Q && U == 1)) {
            if (c.wide) {
                launch_timed(k_sweep<kWideBlock, J, U, VEC4, NT, Q, NC>, dim3(t.nsweep),
                             dim3(kWideBlock), lds, s, tm.start(), score ? nullptr : tm.stop(),
                             t.desc, t.single ? nullptr : t.sweep, step);
                launched = true;
            }
        }
        if (!launched)
            launch_timed(k_sweep<kBlock, J, U, VEC4, NT, Q, NC>, dim3(t.nsweep), dim3(kBlock), lds,
                         s, tm.start(), score ? nullptr : tm.stop(), t.desc,
                         t.single ? nullptr : t.sweep, step);
        FS_HIP(hipGetLastError());
        if (!score) tm.used();
    }
    if (score) {
        launch_timed(k_score<J>, dim3(t.nscore), dim3(kBlock), lds, s,
                     t.nsweep > 0 ? nullptr : tm.start(), tm.stop(), t.desc,
                     t.single ? nullptr : t.score, step);
        FS_HIP(hipGetLastError());
        tm.used();
    }
    return FS_OK;
}

template <int J, int U>
fs_status launch_sweep_ju(const EngineTables &t, const EngineConfig &c, int32_t step, hipStream_t s,
                          TimedLaunch &tm)
{
    if (!c.vec4) return launch_sweep_t<J, 1, false, false, false, 1>(t, c, step, s, tm);
    if (c.queue)
        return c.nt ? launch_sweep_t<J, U, true, true, true, 1>(t, c, step, s, tm)
                    : launch_sweep_t<J, U, true, false, true, 1>(t, c, step, s, tm);
    return c.nt ? launch_sweep_t<J, U, true, true, false, 1>(t, c, step, s, tm)
                : launch_sweep_t<J, U, true, false, false, 1>(t, c, step, s, tm);
}

// Typed launch sets: one load in flight (U = 1), queued or in place, or the
// scalar variant.
template <int J>
fs_status launch_sweep_typed(const EngineTables &t, const EngineConfig &c, int32_t step,
                             hipStream_t s, TimedLaunch &tm)
{
    if (!c.vec4) return launch_sweep_t<J, 1, false, false, false, 2>(t, c, step, s, tm);
    if (c.queue)
        return c.nt ? launch_sweep_t<J, 1, true, true, true, 2>(t, c, step, s, tm)
                    : launch_sweep_t<J, 1, true, false, true, 2>(t, c, step, s, tm);
    return c.nt ? launch_sweep_t<J, 1, true, true, false, 2>(t, c, step, s, tm)
                : launch_sweep_t<J, 1, true, false, false, 2>(t, c, step, s, tm);
}

template <int J>
fs_status launch_sweep_j(const EngineTables &t, const EngineConfig &c, int32_t step, hipStream_t s,
                         TimedLaunch &tm)
{
    if (c.typed) return launch_sweep_typed<J>(t, c, step, s, tm);
    switch (c.U) {
    case 1: return launch_sweep_ju<J, 1>(t, c, step, s, tm);
    case 2: return launch_sweep_ju<J, 2>(t, c, step, s, tm);
    case 4: return launch_sweep_ju<J, 4>(t, c, step, s, tm);
    default: return fail(FS_E_INTERNAL, "unsupported sweep unroll %d", c.U);
    }
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t refresh_lds_bytes(int Kmax) { return 16 * (size_t)(Kmax + 1) + 8 * (size_t)Kmax + 16; }

}  // namespace

// ---------------------------------------------------------------- planning

size_t sweep_lds_of(int J, int Kmax) { return sweep_lds_bytes(J, Kmax); }

int choose_rows_per_group(int32_t nclosed, int32_t M, int64_t total_rows, int32_t K)
{
    // many rows: fewer re-reads of the per-mission state per row; short rows
    // (a few thousand missions) in a launch with rows to spare: enough
    // streaming per workgroup to hide its fixed start-up and scoring latency
    int J = 1;
    if (nclosed >= 2048 || (M < 8192 && nclosed >= 16 && total_rows >= 8192))
        J = 4;
    else if (nclosed >= 1024)
        J = 2;
    J = env_int("FS_SWEEP_J", J);
    if (J != 1 && J != 2 && J != 4 && J != 8 && J != 16) J = 1;
    while (J > 1 && sweep_lds_bytes(J, K) > 56 * 1024) J >>= 1;
    return J;
}

int choose_unroll(int J)
{
    int U = J >= 4 ? 1 : (J >= 2 ? 2 : 4);
    U = env_int("FS_SWEEP_U", U);
    if (U != 1 && U != 2 && U != 4) U = 1;
    return U;
}

InstPlan plan_instance(int32_t B, int32_t M, int32_t K, int J, int target_wg)
{
    InstPlan p;
    const int32_t Mp = (M + 3) / 4 * 4;
    p.nclosed = B - K;
    p.ngroups = p.nclosed > 0 ? (p.nclosed + J - 1) / J : 0;
    int nsplit = 1;
    if (p.ngroups > 0 && target_wg > p.ngroups) {
        nsplit = (target_wg + p.ngroups - 1) / p.ngroups;
        nsplit = std::min(nsplit, std::max(1, Mp / 2048));
    }
    if (p.ngroups > 0) nsplit = env_int("FS_SWEEP_SPLIT", nsplit);
    nsplit = std::max(1, std::min(nsplit, std::max(1, Mp / 4)));
    if (p.ngroups == 0) nsplit = 1;
    int chunk = (Mp + nsplit - 1) / nsplit;
    chunk = (chunk + 3) / 4 * 4;
    p.nsplit = (Mp + chunk - 1) / chunk;
    p.chunk = chunk;
    return p;
}

InstPlan plan_sparse(int32_t B, int32_t M, int32_t K, int target_wg)
{
    InstPlan p;
    const int32_t Mp = (M + 3) / 4 * 4;
    p.sparse = 1;
    p.nclosed = B - K;
    p.ngroups = (B + kSparseW - 1) / kSparseW;
    // mission chunks of at least 1,024 missions; at most target_wg workgroups
    // in all, so that the whole sweep is resident at once (a second, partial
    // round of workgroups would run alone at the end)
    int nsplit = std::max(1, std::max(target_wg, 1) / p.ngroups);
    nsplit = std::min(nsplit, std::max(1, Mp / 1024));
    nsplit = std::max(1, env_int("FS_SPARSE_SPLIT", nsplit));
    int chunk = (Mp + nsplit - 1) / nsplit;
    chunk = (chunk + 63) / 64 * 64;
    p.nsplit = (Mp + chunk - 1) / chunk;
    p.chunk = chunk;
    return p;
}

size_t instance_bytes(int32_t B, int32_t M, int32_t K, const InstPlan &p)
{
    const size_t Mp = (size_t)(M + 3) / 4 * 4;
    const size_t nclosed = (size_t)std::max(p.nclosed, 1);
    size_t n = 0;
    n += align_up(4 * (size_t)K, 256);                          // open list
    n += align_up(4 * nclosed, 256);                            // closed list
    n += align_up(4 * (size_t)K, 256);                          // open tabu expiries
    n += align_up(4 * nclosed, 256);                            // closed tabu expiries
    n += 3 * align_up(4 * (size_t)K, 256);                      // open types, heliport flags,
                                                                // best types
    n += align_up(4 * nclosed, 256);                            // closed heliport flags
    n += align_up(4 * (size_t)B, 256);                          // typed ranking order
    n += 3 * align_up(4 * Mp, 256);                             // b1 b2 o1
    n += 2 * align_up(sizeof(Acc) * kStripes * (K + 1), 256);   // accumulators
    n += align_up(sizeof(Candidate) * std::max(p.ngroups * kScoreParts, 1), 256);
    n += align_up(sizeof(SolveState), 256);
    n += 2 * align_up(4 * (size_t)K, 256);                      // best_open, best_sorted
    if (p.sparse) {
        const size_t lst = (size_t)p.ngroups * kSparseW * Mp;
        const size_t head = (size_t)p.ngroups * kSparseHead * Mp;
        n += align_up(4 * head, 256) + align_up(head, 256);   // sorted heads: costs, ids
        n += align_up(4 * lst, 256) + align_up(lst, 256);     // sorted lists: costs, ids
        n += 2 * align_up(4 * (size_t)B, 256);              // base_slot, base_tabu
        n += align_up(4, 256);                              // wide-cost flag
        if (p.nsplit > 1) {   // the blocks' sums over mission chunks
            const size_t np = (size_t)p.ngroups * kSparseW * (K + 1);
            n += align_up(4 * np, 256) + align_up(8 * np, 256);
        }
    } else if (p.nsplit > 1) {
        const size_t np = (size_t)p.nsplit * p.nclosed * (K + 2);
        n += align_up(4 * np, 256) + align_up(8 * np, 256);
    }
    return n;
}

void carve_instance(InstDesc &d, char *base, int32_t B, int32_t M, int32_t K, const InstPlan &p)
{
    const size_t Mp = (size_t)(M + 3) / 4 * 4;
    const size_t nclosed = (size_t)std::max(p.nclosed, 1);
    char *q = base;
    auto take = [&](size_t bytes) {
        char *r = q;
        q += align_up(bytes, 256);
        return r;
    };
    d.open = (int32_t *)take(4 * (size_t)K);
    d.closed = (int32_t *)take(4 * nclosed);
    d.open_tabu = (int32_t *)take(4 * (size_t)K);
    d.closed_tabu = (int32_t *)take(4 * nclosed);
    d.open_rot = (int32_t *)take(4 * (size_t)K);
    d.open_hel = (int32_t *)take(4 * (size_t)K);
    d.best_rot_sorted = (int32_t *)take(4 * (size_t)K);
    d.closed_hel = (int32_t *)take(4 * nclosed);
    d.rank_order = (int32_t *)take(4 * (size_t)B);
    d.b1 = (int32_t *)take(4 * Mp);
    d.b2 = (int32_t *)take(4 * Mp);
    d.o1 = (int32_t *)take(4 * Mp);
    d.acc[0] = (Acc *)take(sizeof(Acc) * kStripes * (K + 1));
    d.acc[1] = (Acc *)take(sizeof(Acc) * kStripes * (K + 1));
    d.cand = (Candidate *)take(sizeof(Candidate) * std::max(p.ngroups * kScoreParts, 1));
    d.st = (SolveState *)take(sizeof(SolveState));
    d.best_open = (int32_t *)take(4 * (size_t)K);
    d.best_sorted = (int32_t *)take(4 * (size_t)K);
    d.part_cov = nullptr;
    d.part_dist = nullptr;
    d.sparse = p.sparse;
    d.lst_cost = nullptr;
    d.lst_id = nullptr;
    d.base_slot = nullptr;
    d.base_tabu = nullptr;
    d.mm_cost = nullptr;
    d.mm_id = nullptr;
    d.wide = nullptr;
    if (p.sparse) {
        const size_t lst = (size_t)p.ngroups * kSparseW * Mp;
        const size_t head = (size_t)p.ngroups * kSparseHead * Mp;
        d.lst_cost = (int32_t *)take(4 * head);
        d.lst_id = (unsigned char *)take(head);
        d.mm_cost = (int32_t *)take(4 * lst);
        d.mm_id = (unsigned char *)take(lst);
        d.base_slot = (int32_t *)take(4 * (size_t)B);
        d.base_tabu = (int32_t *)take(4 * (size_t)B);
        d.wide = (int32_t *)take(4);
        if (p.nsplit > 1) {
            const size_t np = (size_t)p.ngroups * kSparseW * (K + 1);
            d.part_cov = (int32_t *)take(4 * np);
            d.part_dist = (int64_t *)take(8 * np);
        }
    } else if (p.nsplit > 1) {
        const size_t np = (size_t)p.nsplit * p.nclosed * (K + 2);
        d.part_cov = (int32_t *)take(4 * np);
        d.part_dist = (int64_t *)take(8 * np);
    }
    d.B = B;
    d.M = M;
    d.Mp = (int32_t)Mp;
    d.K = K;
    d.nclosed = p.nclosed;
    d.ngroups = p.ngroups;
    d.ncand = p.sparse && p.nsplit > 1 ? p.ngroups * kScoreParts : p.ngroups;
    d.nsplit = p.nsplit;
    d.chunk = p.chunk;
}

void build_tiles(const std::vector<InstPlan> &plans, const std::vector<int32_t> &Mp,
                 std::vector<Tile> &sweep, std::vector<Tile> &score, std::vector<Tile> &refresh,
                 int refresh_mpt)
{
    sweep.clear();
    score.clear();
    refresh.clear();
    for (size_t i = 0; i < plans.size(); ++i) {
        const InstPlan &p = plans[i];
        const int32_t ng = std::max(p.ngroups, 1);
        for (int32_t g = 0; g < ng; ++g)
            for (int32_t sp = 0; sp < p.nsplit; ++sp) sweep.push_back(Tile{(int32_t)i, g, sp, 0});
        if (p.nsplit > 1)
            for (int32_t g = 0; g < p.ngroups; ++g)
                for (int32_t part = 0; part < (p.sparse ? kScoreParts : 1); ++part)
                    score.push_back(Tile{(int32_t)i, g, part, 0});
        const int32_t nt = (Mp[i] + refresh_mpt - 1) / refresh_mpt;
        for (int32_t g = 0; g < nt; ++g) refresh.push_back(Tile{(int32_t)i, g, 0, 0});
    }
}

// ---------------------------------------------------------------- launches

fs_status engine_reset(const EngineTables &t, int32_t maxB, int32_t Kmax, hipStream_t s)
{
    const int32_t n = std::max(maxB, kStripes * (Kmax + 1));
    const int per = (n + kBlock - 1) / kBlock;
    k_reset<<<t.ninst * per, kBlock, 0, s>>>(t.desc, per);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

fs_status engine_rank_lists(const EngineTables &t, const Tile *row_tiles, int nrow_tiles,
                            int32_t Bmax, hipStream_t s)
{
    if (nrow_tiles > 0) {
        k_rank_rows<<<nrow_tiles, kBlock, 0, s>>>(t.desc, row_tiles);
        FS_HIP(hipGetLastError());
    }
    k_rank_lists<<<t.ninst, kBlock, (size_t)Bmax + 16, s>>>(t.desc);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

fs_status engine_fleet_lists(const EngineTables &t, hipStream_t s)
{
    k_fleet_lists<<<t.ninst, kBlock, 0, s>>>(t.desc);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

namespace {
typedef void (*RefreshKernel)(const InstDesc *, const Tile *, int32_t);

RefreshKernel refresh_kernel(const EngineConfig &c)
{
    if (c.refresh_wide)
        return c.typed ? k_refresh<kBlock, true, kWideBlock> : k_refresh<kBlock, false, kWideBlock>;
    if (c.refresh_mpt == kBlock)
        return c.typed ? k_refresh<kBlock, true> : k_refresh<kBlock, false>;
    return c.typed ? k_refresh<kRefreshMissions, true> : k_refresh<kRefreshMissions, false>;
}
}  // namespace

fs_status engine_init(const EngineTables &t, const EngineConfig &c, int32_t step0, hipStream_t s)
{
    if (t.nrefresh > 0) {
        refresh_kernel(c)<<<t.nrefresh, c.refresh_wide ? kWideBlock : kBlock,
                            refresh_lds_bytes(c.Kmax), s>>>(
            t.desc, t.single ? nullptr : t.refresh, step0);
        FS_HIP(hipGetLastError());
    }
    k_init_score<<<t.ninst, kBlock, 0, s>>>(t.desc);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

namespace {
fs_status sweep_rows(const EngineTables &t, const EngineConfig &c, int32_t step, hipStream_t s)
{
    TimedLaunch timed(0);
    switch (c.J) {
    case 1: return launch_sweep_j<1>(t, c, step, s, timed);
    case 2: return launch_sweep_j<2>(t, c, step, s, timed);
    case 4: return launch_sweep_j<4>(t, c, step, s, timed);
    case 8:
        return c.typed ? launch_sweep_typed<8>(t, c, step, s, timed)
                       : launch_sweep_ju<8, 1>(t, c, step, s, timed);
    case 16:
        // (untyped, in place, one load in flight: the launch set's rule)
        if (c.typed || !c.vec4 || c.queue)
            return fail(FS_E_INTERNAL, "16-row sweep groups need the in-place vector sweep");
        return c.nt ? launch_sweep_t<16, 1, true, true, false, 1>(t, c, step, s, timed)
                    : launch_sweep_t<16, 1, true, false, false, 1>(t, c, step, s, timed);
    default: return fail(FS_E_INTERNAL, "unsupported sweep row count %d", c.J);
    }
}
}  // namespace

fs_status engine_sparse_prepare(const EngineTables &t, EngineConfig &c, hipStream_t s)
{
    // (one instance: the descriptor's plan gives the grid of the list build)
    InstDesc d;
    FS_HIP(hipMemcpyAsync(&d, t.desc, sizeof d, hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    if (!d.sparse) return fail(FS_E_INTERNAL, "sparse preparation of a dense plan");
    const int grid = d.ngroups * ((d.Mp + 63) / 64);
    // packed lists unless some cost does not fit a key (then built again)
    c.sparse_packed = false;
    if (env_int("FS_SPARSE_PACKED", 1) != 0) {
        FS_TRY(engine_fill_i32(d.wide, 1, 0, s));
        k_sparse_build<true><<<grid, kBlock, 0, s>>>(t.desc);
        FS_HIP(hipGetLastError());
        int32_t wide = 1;
        FS_HIP(hipMemcpyAsync(&wide, d.wide, sizeof wide, hipMemcpyDeviceToHost, s));
        FS_HIP(hipStreamSynchronize(s));
        c.sparse_packed = wide == 0;
    }
    if (!c.sparse_packed) {
        k_sparse_build<false><<<grid, kBlock, 0, s>>>(t.desc);
        FS_HIP(hipGetLastError());
    }
    k_sparse_slots<<<std::max(1, std::min(64, (d.B + kBlock - 1) / kBlock)), kBlock, 0, s>>>(
        t.desc);
    FS_HIP(hipGetLastError());
    if (d.nsplit > 1) {   // block sums start at zero; the score kernel clears them after use
        const int64_t np = (int64_t)d.ngroups * kSparseW * (d.K + 1);
        FS_TRY(engine_fill_i32(d.part_cov, np, 0, s));
        FS_TRY(engine_fill_i64(d.part_dist, np, 0, s));
    }
    return FS_OK;
}

namespace {
fs_status sweep_sparse(const EngineTables &t, const EngineConfig &c, int32_t step, hipStream_t s)
{
    const uint32_t lds = (uint32_t)sweep_lds_bytes(kSparseW, c.Kmax);
    {
        TimedLaunch tm(0);
        launch_timed(c.sparse_packed ? k_sweep_sparse<kWideBlock, true>
                                     : k_sweep_sparse<kWideBlock, false>,
                     dim3(t.nsweep), dim3(kWideBlock), lds, s, tm.start(), tm.stop(), t.desc,
                     t.single ? nullptr : t.sweep, step);
        FS_HIP(hipGetLastError());
        tm.used();
    }
    if (t.nscore > 0 && !c.fuse_score) {   // (timed apart, as the "finalize" group)
        TimedLaunch tm(2);
        launch_timed(k_score_sparse<kBlock>, dim3(t.nscore), dim3(kBlock),
                     (uint32_t)sweep_lds_bytes(kSparseW / kScoreParts, c.Kmax), s,
                     tm.start(), tm.stop(), t.desc, t.single ? nullptr : t.score, step);
        FS_HIP(hipGetLastError());
        tm.used();
    }
    return FS_OK;
}
}  // namespace

fs_status engine_sweep(const EngineTables &t, const EngineConfig &c, int32_t step, hipStream_t s)
{
    if (c.sparse) return sweep_sparse(t, c, step, s);
    if (t.nsweep > 0 || t.nscore > 0) FS_TRY(sweep_rows(t, c, step, s));
    if (t.nsweep_tall > 0) {
        EngineTables tall = t;
        tall.sweep = t.sweep_tall;
        tall.nsweep = t.nsweep_tall;
        tall.score = nullptr;
        tall.nscore = 0;
        tall.single = false;   // its own tile table
        EngineConfig ct = c;
        ct.J = c.J_tall;
        ct.U = c.U_tall;
        ct.Kmax = c.Kmax_tall;
        ct.wide = false;
        FS_TRY(sweep_rows(tall, ct, step, s));
    }
    if (t.nsweep_long > 0) {   // (1024-thread workgroups where the form has them)
        EngineTables lng = t;
        lng.sweep = t.sweep_long;
        lng.nsweep = t.nsweep_long;
        lng.score = nullptr;
        lng.nscore = 0;
        lng.single = false;
        EngineConfig cl = c;
        cl.J = c.J_tall;
        cl.U = c.U_tall;
        cl.Kmax = c.Kmax_long;
        cl.wide = true;
        FS_TRY(sweep_rows(lng, cl, step, s));
    }
    return FS_OK;
}

fs_status engine_refresh(const EngineTables &t, const EngineConfig &c, int32_t step, hipStream_t s)
{
    if (t.nrefresh == 0) return FS_OK;
    if (c.fuse_score && t.nscore > 0) {
        // the block scores and the refresh in one launch (timed as "score_refresh")
        typedef void (*Fused)(const InstDesc *, int32_t, int32_t);
        Fused k = c.refresh_wide ? k_score_refresh<kBlock, false, kWideBlock>
                  : c.refresh_mpt == kBlock ? k_score_refresh<kBlock, false, kBlock>
                                            : k_score_refresh<kRefreshMissions, false, kBlock>;
        const uint32_t lds =
            (uint32_t)std::max(refresh_lds_bytes(c.Kmax),
                               sweep_lds_bytes(kSparseW / kScoreParts, c.Kmax));
        TimedLaunch timed(3);
        launch_timed(k, dim3(t.nscore + t.nrefresh), dim3(c.refresh_wide ? kWideBlock : kBlock),
                     lds, s, timed.start(), timed.stop(), t.desc, (int32_t)t.nscore, step);
        FS_HIP(hipGetLastError());
        timed.used();
        return FS_OK;
    }
    TimedLaunch timed(1);
    launch_timed(refresh_kernel(c), dim3(t.nrefresh), dim3(c.refresh_wide ? kWideBlock : kBlock),
                 (uint32_t)refresh_lds_bytes(c.Kmax), s, timed.start(), timed.stop(), t.desc,
                 t.single ? nullptr : t.refresh, step);
    FS_HIP(hipGetLastError());
    timed.used();
    return FS_OK;
}

size_t solo_lds_of(int32_t Mp, int32_t K, int32_t nclosed, int32_t tab_B)
{
    return solo_layout(Mp, K, std::max(nclosed, 1), tab_B).total;
}

fs_status engine_persistent(const EngineTables &t, const EngineConfig &c, hipStream_t s)
{
    if (t.nsolo == 0) return FS_OK;
    TimedLaunch timed(0);
    launch_timed(c.solo_tab ? k_solo<true> : k_solo<false>, dim3(t.nsolo), dim3(kSoloBlock),
                 c.solo_lds, s, timed.start(), timed.stop(), t.desc, t.solo);
    FS_HIP(hipGetLastError());
    timed.used();
    return FS_OK;
}

fs_status engine_outputs(const EngineTables &t, const EngineConfig &c, fs_score *scores,
                         int32_t *errors, hipStream_t s)
{
    (void)c;
    k_outputs<<<t.ninst, kBlock, 0, s>>>(t.desc, scores, errors);
    FS_HIP(hipGetLastError());
    if (t.nrefresh > 0) {
        if (c.refresh_mpt == kBlock)
            k_assign<kBlock><<<t.nrefresh, kBlock, 0, s>>>(t.desc, t.refresh);
        else
            k_assign<kRefreshMissions><<<t.nrefresh, kBlock, 0, s>>>(t.desc, t.refresh);
        FS_HIP(hipGetLastError());
    }
    return FS_OK;
}

fs_status engine_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return FS_OK;
    const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    k_fill_i32<<<grid, kBlock, 0, s>>>(p, n, v);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

fs_status engine_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s)
{
    if (n <= 0) return FS_OK;
    const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    k_fill_i64<<<grid, kBlock, 0, s>>>(p, n, v);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

}  // namespace fs
