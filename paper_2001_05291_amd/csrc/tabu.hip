// Tabu search over swap moves on gfx950 (Section 4.3, Algorithm 3; local-search
// baseline of Section 4.2, Algorithm 2).
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
// Kernels per iteration: k_sweep (streams the closed rows, scores the moves of
// its rows and keeps its best admissible one), k_finalize (one workgroup:
// global argmax, applies the move, tabu list, best-so-far, trace), k_refresh
// (b1/b2/o1 and G, L for the new placement).  All search state lives in device
// memory, so the host only enqueues the same three launches N times.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "fs_internal.h"

namespace fs {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned long long u64;

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ bool better(int32_t ca, int64_t da, int32_t cb, int64_t db)
{
    return ca != cb ? ca > cb : da < db;
}

__device__ __forceinline__ bool cand_better(const Candidate &a, const Candidate &b)
{
    if (!a.valid) return false;
    if (!b.valid) return true;
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

__device__ __forceinline__ Candidate shfl_xor_cand(const Candidate &c, int off)
{
    Candidate o;
    o.valid = __shfl_xor(c.valid, off, 64);
    o.cov = __shfl_xor(c.cov, off, 64);
    o.i_base = __shfl_xor(c.i_base, off, 64);
    o.j_base = __shfl_xor(c.j_base, off, 64);
    o.i_slot = __shfl_xor(c.i_slot, off, 64);
    o.j_slot = __shfl_xor(c.j_slot, off, 64);
    o.dist = __shfl_xor(c.dist, off, 64);
    return o;
}

// Best candidate of the workgroup (a total order, so the result does not
// depend on the reduction order).  Valid in every thread on return.
__device__ Candidate block_best(Candidate c, Candidate *s_red /* kBlock/64 + 1 */)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Candidate o = shfl_xor_cand(c, off);
        if (cand_better(o, c)) c = o;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_red[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        Candidate b = s_red[0];
        for (int w = 1; w < kBlock / 64; ++w)
            if (cand_better(s_red[w], b)) b = s_red[w];
        s_red[kBlock / 64] = b;
    }
    __syncthreads();
    return s_red[kBlock / 64];
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

__global__ __launch_bounds__(kBlock) void k_reset(int32_t *tabu_until, int32_t B, Acc *acc,
                                                  int32_t K, SolveState *st)
{
    const int32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q < B) tabu_until[q] = 0;
    if (q <= K) {
        acc[q].cov = 0;
        acc[q].dist = 0;
    }
    if (q == 0) *st = SolveState{};
}

// ---------------------------------------------------------------- refresh (A2)

// Per mission: nearest and second-nearest open cost, the slot of the nearest
// (lowest base id among equal costs), and the sums G and L_k accumulated into
// acc with integer atomics (exact in any order).
__global__ __launch_bounds__(kBlock) void k_refresh(const int32_t *__restrict__ C, int64_t ldc,
                                                    int32_t M, int32_t Mp, int32_t K, int32_t R,
                                                    const int32_t *__restrict__ open,
                                                    int32_t *__restrict__ b1o,
                                                    int32_t *__restrict__ b2o,
                                                    int32_t *__restrict__ o1o, Acc *__restrict__ acc,
                                                    const SolveState *__restrict__ st)
{
    if (st->stopped) return;
    extern __shared__ __align__(16) unsigned char smem[];
    u64 *s_cov = reinterpret_cast<u64 *>(smem);
    u64 *s_dist = s_cov + (K + 1);
    int32_t *s_open = reinterpret_cast<int32_t *>(s_dist + (K + 1));
    for (int k = threadIdx.x; k <= K; k += kBlock) {
        s_cov[k] = 0;
        s_dist[k] = 0;
    }
    for (int k = threadIdx.x; k < K; k += kBlock) s_open[k] = open[k];
    __syncthreads();

    const int32_t m = blockIdx.x * kBlock + threadIdx.x;
    int32_t g1c = 0, g1d = 0;
    if (m < M) {
        int32_t v1 = INT32_MAX, v2 = INT32_MAX, k1 = 0, id1 = INT32_MAX;
        const int32_t *col = C + m;
#pragma unroll 8
        for (int32_t k = 0; k < K; ++k) {
            const int32_t id = s_open[k];
            const int32_t c = col[(int64_t)id * ldc];
            if (c < v1 || (c == v1 && id < id1)) {
                v2 = v1;
                v1 = c;
                k1 = k;
                id1 = id;
            } else if (c < v2) {
                v2 = c;
            }
        }
        b1o[m] = v1;
        b2o[m] = v2;
        o1o[m] = k1;
        g1c = v1 <= R;
        g1d = g1c ? v1 : 0;
        const int32_t g2c = v2 <= R;
        const int32_t g2d = g2c ? v2 : 0;
        const int32_t dc = g2c - g1c, dd = g2d - g1d;
        if (dc | dd) {
            atomicAdd(&s_cov[1 + k1], (u64)(int64_t)dc);
            atomicAdd(&s_dist[1 + k1], (u64)(int64_t)dd);
        }
    } else if (m < Mp) {
        // padding missions: a sentinel below every cost, so the sweep skips them
        b1o[m] = INT32_MIN;
        b2o[m] = INT32_MIN;
        o1o[m] = 0;
    }
    const int32_t wc = wave_sum_i32(g1c);
    const int64_t wd = wave_sum_i64((int64_t)g1d);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&s_cov[0], (u64)(int64_t)wc);
        atomicAdd(&s_dist[0], (u64)wd);
    }
    __syncthreads();
    for (int k = threadIdx.x; k <= K; k += kBlock) {
        const u64 c = s_cov[k], d = s_dist[k];
        if (c | d) {
            atomicAdd(&acc[k].cov, c);
            atomicAdd(&acc[k].dist, d);
        }
    }
}

// cur = best = G of the initial placement; best_open = open.
__global__ __launch_bounds__(kBlock) void k_init_score(const Acc *__restrict__ acc,
                                                       SolveState *__restrict__ st,
                                                       const int32_t *__restrict__ open,
                                                       int32_t *__restrict__ best_open, int32_t K)
{
    if (threadIdx.x == 0) {
        SolveState s{};
        s.cur_cov = (int32_t)acc[0].cov;
        s.cur_dist = (int64_t)acc[0].dist;
        s.best_cov = s.cur_cov;
        s.best_dist = s.cur_dist;
        *st = s;
    }
    for (int k = threadIdx.x; k < K; k += kBlock) best_open[k] = open[k];
}

// ---------------------------------------------------------------- sweep (A3, A4 local)

struct SweepArgs {
    const int32_t *C;
    int64_t ldc;
    int32_t B, M, Mp, K, R, mode;
    int32_t nclosed, chunk, nsplit, ngroups;
    const int32_t *open, *closed;
    const int32_t *b1, *b2, *o1;
    const Acc *acc;
    const int32_t *tabu_until;
    const SolveState *st;
    Candidate *cand;
    int32_t *sc_cov;
    int64_t *sc_dist;
    int32_t *part_cov;
    int64_t *part_dist;
};

__device__ __forceinline__ void visit(int32_t c, int32_t b1, int32_t b2, int32_t o1, int32_t g1c,
                                      int32_t g1d, int32_t g2c, int32_t g2d, int32_t R,
                                      int32_t &t1c, int64_t &t1d, int32_t *__restrict__ bc,
                                      u64 *__restrict__ bd)
{
    if (c < b2) {
        const int32_t v1 = min(c, b1);
        const int32_t u = max(c, b1);
        const int32_t cv = v1 <= R;
        t1c += cv - g1c;
        t1d += (int64_t)((cv ? v1 : 0) - g1d);
        const int32_t cu = u <= R;
        const int32_t dc = cu - g2c;
        const int32_t dd = (cu ? u : 0) - g2d;
        if (dc | dd) {
            atomicAdd(bc + o1, dc);
            atomicAdd(bd + o1, (u64)(int64_t)dd);
        }
    }
}

// Scores of the J x K moves of a row group from summed T1 (per row) and bins
// (per row and out-slot); writes the optional full score table and the best
// admissible candidate of the group.
template <int J>
__device__ void score_group(const SweepArgs &a, int32_t g, const int32_t *s_jrow,
                            const int32_t *s_open, const int32_t *t1c, const int64_t *t1d,
                            const int32_t *bc, const u64 *bd, Candidate *s_red)
{
    const SolveState *st = a.st;
    const int32_t t = st->t + 1;
    const int32_t cur_c = st->cur_cov, best_c = st->best_cov;
    const int64_t cur_d = st->cur_dist, best_d = st->best_dist;
    const int32_t Gc = (int32_t)a.acc[0].cov;
    const int64_t Gd = (int64_t)a.acc[0].dist;
    const int32_t K = a.K;
    Candidate mine{};
    for (int32_t idx = threadIdx.x; idx < J * K; idx += kBlock) {
        const int32_t r = idx / K, k = idx - r * K;
        const int32_t js = g * J + r;
        if (js >= a.nclosed) continue;
        const int32_t cov = Gc + (int32_t)a.acc[1 + k].cov + t1c[r] + bc[idx];
        const int64_t dist = Gd + (int64_t)a.acc[1 + k].dist + t1d[r] + (int64_t)bd[idx];
        const int32_t i = s_open[k], j = s_jrow[r];
        if (a.sc_cov) {
            a.sc_cov[(int64_t)k * a.B + j] = cov;
            a.sc_dist[(int64_t)k * a.B + j] = dist;
        }
        bool adm;
        if (a.mode == 1)
            adm = better(cov, dist, cur_c, cur_d);
        else
            adm = (a.tabu_until[i] < t && a.tabu_until[j] < t) || better(cov, dist, best_c, best_d);
        if (adm) {
            Candidate c;
            c.valid = 1;
            c.cov = cov;
            c.dist = dist;
            c.i_base = i;
            c.j_base = j;
            c.i_slot = k;
            c.j_slot = js;
            if (cand_better(c, mine)) mine = c;
        }
    }
    mine = block_best(mine, s_red);
    if (threadIdx.x == 0) a.cand[g] = mine;
}

// One workgroup = J closed rows x one mission chunk.  With a single chunk the
// workgroup also scores its moves (FUSED); otherwise it writes its partial
// sums and k_score finishes the group.  Block ids are mapped chunk-minor so
// that consecutive ids (which the dispatcher spreads over the 8 XCDs) split
// the mission axis: each XCD's L2 then holds only its chunks' b1/b2/o1.
template <int J, bool VEC4, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs a)
{
    if (a.st->stopped) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t K = a.K;
    u64 *bd = reinterpret_cast<u64 *>(smem);                         // J*K
    int32_t *bc = reinterpret_cast<int32_t *>(bd + J * K);           // J*K
    int32_t *s_open = bc + J * K;                                    // K
    __shared__ int32_t s_jrow[J];
    __shared__ int32_t s_t1c[kBlock / 64][J];
    __shared__ int64_t s_t1d[kBlock / 64][J];
    __shared__ int32_t s_sum_c[J];
    __shared__ int64_t s_sum_d[J];
    __shared__ Candidate s_red[kBlock / 64 + 1];

    const int32_t bid = blockIdx.x;
    const int32_t sp = bid % a.nsplit;
    const int32_t g = bid / a.nsplit;
    for (int q = threadIdx.x; q < J * K; q += kBlock) {
        bd[q] = 0;
        bc[q] = 0;
    }
    if (FUSED)
        for (int q = threadIdx.x; q < K; q += kBlock) s_open[q] = a.open[q];
    if (threadIdx.x < J) {
        const int32_t js = g * J + threadIdx.x;
        s_jrow[threadIdx.x] = a.closed[js < a.nclosed ? js : 0];
    }
    __syncthreads();

    int32_t jrow[J];
#pragma unroll
    for (int r = 0; r < J; ++r) jrow[r] = s_jrow[r];
    int32_t t1c[J];
    int64_t t1d[J];
#pragma unroll
    for (int r = 0; r < J; ++r) {
        t1c[r] = 0;
        t1d[r] = 0;
    }
    const int32_t R = a.R;
    const int32_t m0 = sp * a.chunk;
    const int32_t m1 = min(a.Mp, m0 + a.chunk);

    if (VEC4) {
        const v4i *b1v = reinterpret_cast<const v4i *>(a.b1);
        const v4i *b2v = reinterpret_cast<const v4i *>(a.b2);
        const v4i *o1v = reinterpret_cast<const v4i *>(a.o1);
        const v4i *rows[J];
#pragma unroll
        for (int r = 0; r < J; ++r)
            rows[r] = reinterpret_cast<const v4i *>(a.C + (int64_t)jrow[r] * a.ldc);
        for (int32_t q = (m0 >> 2) + threadIdx.x; q < (m1 >> 2); q += kBlock) {
            v4i cv[J];
#pragma unroll
            for (int r = 0; r < J; ++r) cv[r] = __builtin_nontemporal_load(rows[r] + q);
            const v4i vb1 = b1v[q], vb2 = b2v[q], vo1 = o1v[q];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int32_t b1 = vb1[e], b2 = vb2[e], o1 = vo1[e];
                const int32_t g1c = b1 <= R, g1d = g1c ? b1 : 0;
                const int32_t g2c = b2 <= R, g2d = g2c ? b2 : 0;
#pragma unroll
                for (int r = 0; r < J; ++r)
                    visit(cv[r][e], b1, b2, o1, g1c, g1d, g2c, g2d, R, t1c[r], t1d[r], bc + r * K,
                          bd + r * K);
            }
        }
    } else {
        const int32_t mend = min(m1, a.M);
        for (int32_t m = m0 + threadIdx.x; m < mend; m += kBlock) {
            int32_t cv[J];
#pragma unroll
            for (int r = 0; r < J; ++r) cv[r] = a.C[(int64_t)jrow[r] * a.ldc + m];
            const int32_t b1 = a.b1[m], b2 = a.b2[m], o1 = a.o1[m];
            const int32_t g1c = b1 <= R, g1d = g1c ? b1 : 0;
            const int32_t g2c = b2 <= R, g2d = g2c ? b2 : 0;
#pragma unroll
            for (int r = 0; r < J; ++r)
                visit(cv[r], b1, b2, o1, g1c, g1d, g2c, g2d, R, t1c[r], t1d[r], bc + r * K,
                      bd + r * K);
        }
    }

    // per-row sums of the common term across the workgroup
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < J; ++r) {
        const int32_t c = wave_sum_i32(t1c[r]);
        const int64_t d = wave_sum_i64(t1d[r]);
        if (lane == 0) {
            s_t1c[wave][r] = c;
            s_t1d[wave][r] = d;
        }
    }
    __syncthreads();
    if (threadIdx.x < J) {
        int32_t c = 0;
        int64_t d = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            c += s_t1c[w][threadIdx.x];
            d += s_t1d[w][threadIdx.x];
        }
        s_sum_c[threadIdx.x] = c;
        s_sum_d[threadIdx.x] = d;
    }
    __syncthreads();

    if (FUSED) {
        score_group<J>(a, g, s_jrow, s_open, s_sum_c, s_sum_d, bc, bd, s_red);
    } else {
        // partial sums of this chunk: [T1, bin_0 .. bin_{K-1}] per row
        const int32_t K1 = K + 1;
        for (int32_t idx = threadIdx.x; idx < J * K1; idx += kBlock) {
            const int32_t r = idx / K1, k = idx - r * K1;
            const int32_t js = g * J + r;
            if (js >= a.nclosed) continue;
            const int64_t at = ((int64_t)sp * a.nclosed + js) * K1 + k;
            if (k == 0) {
                a.part_cov[at] = s_sum_c[r];
                a.part_dist[at] = s_sum_d[r];
            } else {
                a.part_cov[at] = bc[r * K + k - 1];
                a.part_dist[at] = (int64_t)bd[r * K + k - 1];
            }
        }
    }
}

// Sums the chunk partials of one row group and scores its moves.
template <int J>
__global__ __launch_bounds__(kBlock) void k_score(SweepArgs a)
{
    if (a.st->stopped) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t K = a.K, K1 = K + 1;
    u64 *bd = reinterpret_cast<u64 *>(smem);
    int32_t *bc = reinterpret_cast<int32_t *>(bd + J * K);
    int32_t *s_open = bc + J * K;
    __shared__ int32_t s_jrow[J];
    __shared__ int32_t s_sum_c[J];
    __shared__ int64_t s_sum_d[J];
    __shared__ Candidate s_red[kBlock / 64 + 1];
    const int32_t g = blockIdx.x;
    for (int q = threadIdx.x; q < K; q += kBlock) s_open[q] = a.open[q];
    if (threadIdx.x < J) {
        const int32_t js = g * J + threadIdx.x;
        s_jrow[threadIdx.x] = a.closed[js < a.nclosed ? js : 0];
    }
    for (int32_t idx = threadIdx.x; idx < J * K1; idx += kBlock) {
        const int32_t r = idx / K1, k = idx - r * K1;
        const int32_t js = g * J + r;
        int32_t c = 0;
        int64_t d = 0;
        if (js < a.nclosed) {
            for (int32_t sp = 0; sp < a.nsplit; ++sp) {
                const int64_t at = ((int64_t)sp * a.nclosed + js) * K1 + k;
                c += a.part_cov[at];
                d += a.part_dist[at];
            }
        }
        if (k == 0) {
            s_sum_c[r] = c;
            s_sum_d[r] = d;
        } else {
            bc[r * K + k - 1] = c;
            bd[r * K + k - 1] = (u64)d;
        }
    }
    __syncthreads();
    score_group<J>(a, g, s_jrow, s_open, s_sum_c, s_sum_d, bc, bd, s_red);
}

// ---------------------------------------------------------------- finalize (A4, A5)

struct FinalArgs {
    const Candidate *cand;
    int32_t ncand, K, T, mode;
    int32_t *open, *closed, *tabu_until;
    SolveState *st;
    Acc *acc;
    int32_t *best_open;
    fs_trace_rec *trace;
};

__global__ __launch_bounds__(kBlock) void k_finalize(FinalArgs a)
{
    __shared__ Candidate s_red[kBlock / 64 + 1];
    __shared__ int32_t s_improved;
    SolveState *st = a.st;
    const int32_t stopped = st->stopped;
    Candidate best{};
    if (!stopped)
        for (int32_t q = threadIdx.x; q < a.ncand; q += kBlock) {
            const Candidate c = a.cand[q];
            if (cand_better(c, best)) best = c;
        }
    if (threadIdx.x == 0) s_improved = 0;
    best = block_best(best, s_red);  // contains barriers

    if (threadIdx.x == 0) {
        const int32_t t = st->t + 1;
        int32_t moved = 0;
        if (!stopped) {
            // the refreshed value of the current placement must equal the
            // score the executed move was chosen with
            if ((int32_t)a.acc[0].cov != st->cur_cov || (int64_t)a.acc[0].dist != st->cur_dist) {
                if (!st->error) {
                    st->error = 1;
                    st->err_iter = t;
                }
            }
            if (best.valid) {
                a.open[best.i_slot] = best.j_base;
                a.closed[best.j_slot] = best.i_base;
                a.tabu_until[best.i_base] = t + a.T;
                a.tabu_until[best.j_base] = t + a.T;
                st->cur_cov = best.cov;
                st->cur_dist = best.dist;
                moved = 1;
                if (better(best.cov, best.dist, st->best_cov, st->best_dist)) {
                    st->best_cov = best.cov;
                    st->best_dist = best.dist;
                    st->best_iter = t;
                    s_improved = 1;
                }
            } else if (a.mode == 1) {
                st->stopped = 1;
            }
        }
        if (a.trace) {
            fs_trace_rec rec;
            rec.iter = t;
            rec.out_base = moved ? best.i_base : -1;
            rec.in_base = moved ? best.j_base : -1;
            rec.moved = moved;
            rec.cur_cov = st->cur_cov;
            rec.best_cov = st->best_cov;
            rec.cur_dist = st->cur_dist;
            rec.best_dist = st->best_dist;
            a.trace[t - 1] = rec;
        }
        st->t = t;
    }
    __syncthreads();
    if (s_improved)
        for (int32_t k = threadIdx.x; k < a.K; k += kBlock) a.best_open[k] = a.open[k];
    if (!stopped)
        for (int32_t k = threadIdx.x; k <= a.K; k += kBlock) {
            a.acc[k].cov = 0;
            a.acc[k].dist = 0;
        }
}

// ---------------------------------------------------------------- assignment

// Nearest open base of each mission (open ids ascending, so the first strict
// minimum is the lowest id among equal costs), or -1 beyond R.
__global__ __launch_bounds__(kBlock) void k_assign(const int32_t *__restrict__ C, int64_t ldc,
                                                   int32_t M, const int32_t *__restrict__ open,
                                                   int32_t K, int32_t R,
                                                   int32_t *__restrict__ out)
{
    const int32_t m = blockIdx.x * kBlock + threadIdx.x;
    if (m >= M) return;
    int32_t v = INT32_MAX, who = -1;
    for (int32_t k = 0; k < K; ++k) {
        const int32_t id = open[k];
        const int32_t c = C[(int64_t)id * ldc + m];
        if (c < v) {
            v = c;
            who = id;
        }
    }
    out[m] = v <= R ? who : -1;
}

// ---------------------------------------------------------------- launch helpers

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    return atoi(v);
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t sweep_lds(int J, int K) { return (size_t)J * K * 12 + (size_t)K * 4; }

template <int J, bool VEC4, bool FUSED>
fs_status launch_sweep_t(const SweepArgs &a, hipStream_t s)
{
    const int grid = a.ngroups * a.nsplit;
    k_sweep<J, VEC4, FUSED><<<grid, kBlock, sweep_lds(J, a.K), s>>>(a);
    FS_HIP(hipGetLastError());
    if (!FUSED) {
        k_score<J><<<a.ngroups, kBlock, sweep_lds(J, a.K), s>>>(a);
        FS_HIP(hipGetLastError());
    }
    return FS_OK;
}

template <int J>
fs_status launch_sweep_j(const SweepArgs &a, bool vec4, hipStream_t s)
{
    const bool fused = a.nsplit == 1;
    if (vec4)
        return fused ? launch_sweep_t<J, true, true>(a, s) : launch_sweep_t<J, true, false>(a, s);
    return fused ? launch_sweep_t<J, false, true>(a, s) : launch_sweep_t<J, false, false>(a, s);
}

}  // namespace

// ---------------------------------------------------------------- planning

SweepPlan plan_sweep(const Problem &pb)
{
    SweepPlan p;
    const int32_t nclosed = pb.B - pb.K;
    p.vec4 = (pb.ldc % 4 == 0) && ((uintptr_t)pb.C % 16 == 0);
    int J = 1;
    if (nclosed >= 8192)
        J = 4;
    else if (nclosed >= 2048)
        J = 2;
    J = env_int("FS_SWEEP_J", J);
    if (J != 1 && J != 2 && J != 4 && J != 8) J = 1;
    while (J > 1 && (size_t)J * pb.K * 12 > 48 * 1024) J >>= 1;
    p.J = J;
    p.ngroups = nclosed > 0 ? (nclosed + J - 1) / J : 0;
    // enough workgroups to fill 256 CUs several times over, chunks of >= 2048 missions
    int nsplit = 1;
    if (p.ngroups > 0) {
        const int target = env_int("FS_SWEEP_TARGET_WG", 2048);
        nsplit = (target + p.ngroups - 1) / p.ngroups;
        const int max_split = std::max(1, pb.Mp / 2048);
        nsplit = std::min(nsplit, max_split);
        nsplit = env_int("FS_SWEEP_SPLIT", nsplit);
        nsplit = std::max(1, std::min(nsplit, std::max(1, pb.Mp / 4)));
    }
    int chunk = (pb.Mp + nsplit - 1) / nsplit;
    chunk = (chunk + 3) / 4 * 4;
    nsplit = (pb.Mp + chunk - 1) / chunk;
    p.nsplit = nsplit;
    p.chunk = chunk;
    p.ncand = p.ngroups;
    return p;
}

size_t workspace_bytes(const Problem &pb, const SweepPlan &plan)
{
    const size_t K = pb.K, B = pb.B, Mp = pb.Mp, nclosed = pb.B - pb.K;
    size_t n = 0;
    n += align_up(4 * K, 256);                      // open
    n += align_up(4 * std::max<size_t>(nclosed, 1), 256);
    n += align_up(4 * B, 256);                      // tabu_until
    n += 3 * align_up(4 * Mp, 256);                 // b1 b2 o1
    n += align_up(sizeof(Acc) * (K + 1), 256);
    n += align_up(sizeof(Candidate) * std::max(plan.ncand, 1), 256);
    n += align_up(sizeof(SolveState), 256);
    n += align_up(4 * K, 256);                      // best_open
    if (plan.nsplit > 1) {
        const size_t np = (size_t)plan.nsplit * nclosed * (K + 1);
        n += align_up(4 * np, 256) + align_up(8 * np, 256);
    }
    return n;
}

void carve_workspace(Workspace &ws, void *base, const Problem &pb, const SweepPlan &plan)
{
    const size_t K = pb.K, B = pb.B, Mp = pb.Mp, nclosed = pb.B - pb.K;
    char *p = (char *)base;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += align_up(bytes, 256);
        return q;
    };
    ws.base = base;
    ws.open = (int32_t *)take(4 * K);
    ws.closed = (int32_t *)take(4 * std::max<size_t>(nclosed, 1));
    ws.tabu_until = (int32_t *)take(4 * B);
    ws.b1 = (int32_t *)take(4 * Mp);
    ws.b2 = (int32_t *)take(4 * Mp);
    ws.o1 = (int32_t *)take(4 * Mp);
    ws.acc = (Acc *)take(sizeof(Acc) * (K + 1));
    ws.cand = (Candidate *)take(sizeof(Candidate) * std::max(plan.ncand, 1));
    ws.st = (SolveState *)take(sizeof(SolveState));
    ws.best_open = (int32_t *)take(4 * K);
    if (plan.nsplit > 1) {
        const size_t np = (size_t)plan.nsplit * nclosed * (K + 1);
        ws.part_cov = (int32_t *)take(4 * np);
        ws.part_dist = (int64_t *)take(8 * np);
    }
    ws.bytes = (size_t)(p - (char *)base);
}

// ---------------------------------------------------------------- launches

fs_status launch_setup(const Problem &pb, const SweepPlan &plan, const Workspace &ws,
                       const int32_t *open_host, hipStream_t s)
{
    (void)plan;
    const int32_t B = pb.B, K = pb.K;
    // closed list: the complement of the open set, ascending id
    std::vector<unsigned char> in(B, 0);
    for (int32_t k = 0; k < K; ++k) in[open_host[k]] = 1;
    std::vector<int32_t> closed;
    closed.reserve(B - K);
    for (int32_t b = 0; b < B; ++b)
        if (!in[b]) closed.push_back(b);
    FS_HIP(hipMemcpyAsync(ws.open, open_host, 4 * (size_t)K, hipMemcpyHostToDevice, s));
    if (!closed.empty())
        FS_HIP(hipMemcpyAsync(ws.closed, closed.data(), 4 * closed.size(), hipMemcpyHostToDevice, s));
    // the copies above are from pageable memory: HIP stages them before
    // returning, so the vector may go out of scope afterwards
    FS_HIP(hipStreamSynchronize(s));
    const int32_t n = std::max(B, K + 1);
    k_reset<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(ws.tabu_until, B, ws.acc, K, ws.st);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

fs_status launch_refresh(const Problem &pb, const Workspace &ws, hipStream_t s)
{
    const size_t lds = 16 * (size_t)(pb.K + 1) + 4 * (size_t)pb.K;
    TimedLaunch timed(1, s);
    k_refresh<<<(pb.Mp + kBlock - 1) / kBlock, kBlock, lds, s>>>(
        pb.C, pb.ldc, pb.M, pb.Mp, pb.K, pb.R, ws.open, ws.b1, ws.b2, ws.o1, ws.acc, ws.st);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

fs_status launch_init_score(const Problem &pb, const Workspace &ws, hipStream_t s)
{
    k_init_score<<<1, kBlock, 0, s>>>(ws.acc, ws.st, ws.open, ws.best_open, pb.K);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

fs_status launch_sweep(const Problem &pb, const SweepPlan &plan, const Workspace &ws,
                       int32_t *sc_cov, int64_t *sc_dist, hipStream_t s)
{
    if (plan.ngroups == 0) return FS_OK;
    TimedLaunch timed(0, s);
    SweepArgs a;
    a.C = pb.C;
    a.ldc = pb.ldc;
    a.B = pb.B;
    a.M = pb.M;
    a.Mp = pb.Mp;
    a.K = pb.K;
    a.R = pb.R;
    a.mode = pb.mode;
    a.nclosed = pb.B - pb.K;
    a.chunk = plan.chunk;
    a.nsplit = plan.nsplit;
    a.ngroups = plan.ngroups;
    a.open = ws.open;
    a.closed = ws.closed;
    a.b1 = ws.b1;
    a.b2 = ws.b2;
    a.o1 = ws.o1;
    a.acc = ws.acc;
    a.tabu_until = ws.tabu_until;
    a.st = ws.st;
    a.cand = ws.cand;
    a.sc_cov = sc_cov;
    a.sc_dist = sc_dist;
    a.part_cov = ws.part_cov;
    a.part_dist = ws.part_dist;
    switch (plan.J) {
    case 1: return launch_sweep_j<1>(a, plan.vec4, s);
    case 2: return launch_sweep_j<2>(a, plan.vec4, s);
    case 4: return launch_sweep_j<4>(a, plan.vec4, s);
    case 8: return launch_sweep_j<8>(a, plan.vec4, s);
    default: return fail(FS_E_INTERNAL, "unsupported sweep row count %d", plan.J);
    }
}

fs_status launch_finalize(const Problem &pb, const SweepPlan &plan, const Workspace &ws,
                          fs_trace_rec *trace, hipStream_t s)
{
    FinalArgs a;
    a.cand = ws.cand;
    a.ncand = plan.ncand;
    a.K = pb.K;
    a.T = pb.T;
    a.mode = pb.mode;
    a.open = ws.open;
    a.closed = ws.closed;
    a.tabu_until = ws.tabu_until;
    a.st = ws.st;
    a.acc = ws.acc;
    a.best_open = ws.best_open;
    a.trace = trace;
    TimedLaunch timed(2, s);
    k_finalize<<<1, kBlock, 0, s>>>(a);
    FS_HIP(hipGetLastError());
    return FS_OK;
}

// ---------------------------------------------------------------- validation

namespace {

fs_status check_problem(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                        int32_t R, Problem &pb)
{
    FS_TRY(check_table(C, ldc, B, M));
    if (K < 1 || K > B) return fail(FS_E_INVALID, "K=%d must be in [1, B=%d]", K, B);
    if (K > kMaxK) return fail(FS_E_INVALID, "K=%d exceeds the supported %d vehicles", K, kMaxK);
    if (R < 0 || R == INT32_MAX) return fail(FS_E_INVALID, "range %d outside [0, INT32_MAX)", R);
    if ((int64_t)M + 3 > INT32_MAX) return fail(FS_E_INVALID, "M=%d too large", M);
    pb.C = C;
    pb.ldc = ldc;
    pb.B = B;
    pb.M = M;
    pb.K = K;
    pb.R = R;
    pb.T = 0;
    pb.N = 0;
    pb.mode = 0;
    pb.Mp = (M + 3) / 4 * 4;
    return FS_OK;
}

// Device-resident list of K ids -> host, validated.
fs_status fetch_open_list(const int32_t *dev, int32_t K, int32_t B, std::vector<int32_t> &out,
                          hipStream_t s)
{
    out.assign(K, 0);
    FS_HIP(hipMemcpyAsync(out.data(), dev, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    return check_open_list(out, B);
}

struct DeviceBuffer {
    void *p = nullptr;
    hipStream_t s = nullptr;
    ~DeviceBuffer()
    {
        if (p) (void)hipFreeAsync(p, s);
    }
};

}  // namespace

}  // namespace fs

// ---------------------------------------------------------------- entry points

extern "C" fs_status fs_move_scores(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                                    const int32_t *open, int32_t K, int32_t range_m,
                                    int32_t *cov_out, int64_t *dist_out, void *stream)
{
    using namespace fs;
    Problem pb;
    FS_TRY(check_problem(C, ldc, B, M, K, range_m, pb));
    if (!open || !cov_out || !dist_out) return fail(FS_E_INVALID, "NULL open or output pointer");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> ids;
    FS_TRY(fetch_open_list(open, K, B, ids, s));
    const SweepPlan plan = plan_sweep(pb);
    DeviceBuffer buf;
    buf.s = s;
    FS_HIP(hipMallocAsync(&buf.p, workspace_bytes(pb, plan), s));
    Workspace ws;
    carve_workspace(ws, buf.p, pb, plan);
    const int64_t n = (int64_t)K * B;
    const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    k_fill_i32<<<grid, kBlock, 0, s>>>(cov_out, n, -1);
    FS_HIP(hipGetLastError());
    k_fill_i64<<<grid, kBlock, 0, s>>>(dist_out, n, -1);
    FS_HIP(hipGetLastError());
    FS_TRY(launch_setup(pb, plan, ws, ids.data(), s));
    FS_TRY(launch_refresh(pb, ws, s));
    FS_TRY(launch_init_score(pb, ws, s));
    FS_TRY(launch_sweep(pb, plan, ws, cov_out, dist_out, s));
    FS_HIP(hipStreamSynchronize(s));
    return FS_OK;
}

extern "C" fs_status fs_tabu_solve(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                                   const fs_params *p, const int32_t *init_open,
                                   int32_t *best_open_out, fs_score *score_out,
                                   int32_t *assign_out, fs_trace_rec *trace_out, void *stream)
{
    using namespace fs;
    if (!p) return fail(FS_E_INVALID, "params pointer is NULL");
    Problem pb;
    FS_TRY(check_problem(C, ldc, B, M, K, p->range_m, pb));
    if (p->tenure < 0) return fail(FS_E_INVALID, "tenure %d < 0", p->tenure);
    if (p->iterations < 0) return fail(FS_E_INVALID, "iterations %d < 0", p->iterations);
    if ((int64_t)p->iterations + p->tenure >= INT32_MAX)
        return fail(FS_E_INVALID, "iterations + tenure overflow int32");
    if (p->mode != 0 && p->mode != 1) return fail(FS_E_INVALID, "mode %d not 0 or 1", p->mode);
    if (!best_open_out || !score_out) return fail(FS_E_INVALID, "NULL output pointer");
    pb.T = p->tenure;
    pb.N = p->iterations;
    pb.mode = p->mode;
    hipStream_t s = (hipStream_t)stream;

    std::vector<int32_t> init;
    if (init_open) {
        FS_TRY(fetch_open_list(init_open, K, B, init, s));
    } else {
        DeviceBuffer rk;
        rk.s = s;
        FS_HIP(hipMallocAsync(&rk.p, 8 * (size_t)B + 4 * (size_t)K, s));
        int64_t *sums = (int64_t *)rk.p;
        int32_t *order = (int32_t *)(sums + B);
        FS_TRY(launch_rank(C, ldc, B, M, K, order, sums, s));
        init.assign(K, 0);
        FS_HIP(hipMemcpyAsync(init.data(), order, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
        FS_HIP(hipStreamSynchronize(s));
        std::sort(init.begin(), init.end());
    }

    const SweepPlan plan = plan_sweep(pb);
    DeviceBuffer buf;
    buf.s = s;
    FS_HIP(hipMallocAsync(&buf.p, workspace_bytes(pb, plan), s));
    Workspace ws;
    carve_workspace(ws, buf.p, pb, plan);
    FS_TRY(launch_setup(pb, plan, ws, init.data(), s));
    FS_TRY(launch_refresh(pb, ws, s));
    FS_TRY(launch_init_score(pb, ws, s));
    for (int32_t t = 1; t <= pb.N; ++t) {
        FS_TRY(launch_sweep(pb, plan, ws, nullptr, nullptr, s));
        FS_TRY(launch_finalize(pb, plan, ws, trace_out, s));
        if (t < pb.N) FS_TRY(launch_refresh(pb, ws, s));
    }

    SolveState h{};
    std::vector<int32_t> best(K);
    FS_HIP(hipMemcpyAsync(&h, ws.st, sizeof h, hipMemcpyDeviceToHost, s));
    FS_HIP(hipMemcpyAsync(best.data(), ws.best_open, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    std::sort(best.begin(), best.end());
    FS_HIP(hipMemcpyAsync(best_open_out, best.data(), 4 * (size_t)K, hipMemcpyHostToDevice, s));
    if (assign_out) {
        FS_HIP(hipMemcpyAsync(ws.open, best.data(), 4 * (size_t)K, hipMemcpyHostToDevice, s));
        k_assign<<<(M + kBlock - 1) / kBlock, kBlock, 0, s>>>(C, ldc, M, ws.open, K, pb.R,
                                                             assign_out);
        FS_HIP(hipGetLastError());
    }
    FS_HIP(hipStreamSynchronize(s));
    if (h.error)
        return fail(FS_E_INTERNAL, "refreshed placement value disagrees with the move score at "
                                   "iteration %d", h.err_iter);
    score_out->coverage = h.best_cov;
    score_out->best_iter = h.best_iter;
    score_out->distance = h.best_dist;
    return FS_OK;
}
