/*
 * perm_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * The paper's stochastic searches (Section 4.2-4.3, Algorithms 2 and 3 with
 * their Permutation_a / Permutation_b scan orders), as a plain CPU reference
 * for the permuted-search modes of the HIP path.  Same status and rules as
 * fleetstage_oracle.c: loaded only by the tests, the smoke check and the
 * benchmark's CPU baseline; shares no code with the HIP path.
 *
 * Readings of the paper followed here:
 *   - With moves read as base swaps, the two random mission orders of the
 *     paper become one random order over the swap moves.  Each pass draws a
 *     fresh order: move (i, j) (base i leaves, base j enters) has priority
 *     pi_p(i, j) = mix64(z_p + (i * B + j + 1) * GAMMA) with
 *     z_p = mix64(seed + (p + 1) * GAMMA), mix64 being the SplitMix64 output
 *     function (Steele, Lea and Flood, OOPSLA 2014).  For fixed z_p the map
 *     (i, j) -> pi is injective, so the order is a permutation.
 *   - A pass scans the moves of the current placement in ascending priority,
 *     continuing after the last accepted move, and accepts the first one that
 *     strictly improves the current placement (Section 4.3 accepts improving
 *     changes only); in the Tabu variant a move touching a tabu base is
 *     skipped (both bases of an accepted move stay tabu through iteration
 *     t + T, as in reading 11).  When the scan reaches the end of the order,
 *     a new pass starts if this pass accepted a move, else the search stops.
 *   - One iteration is one scan to the next acceptance (a move) or to the end
 *     of the order (no move: a new pass starts, or the search stops and every
 *     later iteration is a no-move record).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void fso_rank_bases(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                    int32_t *open_out, int32_t *order_out, int64_t *sums_out);
void fso_placement_value(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                         const int32_t *S, int32_t K, int32_t R,
                         int32_t *cov_out, int64_t *dist_out);

#define FSO_GAMMA 0x9E3779B97F4A7C15ull

/* SplitMix64 output function. */
uint64_t fso_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Priority of move (i, j) in pass p of a search seeded with `seed`. */
uint64_t fso_perm_priority(uint64_t seed, int32_t pass, int32_t B, int32_t i, int32_t j)
{
    const uint64_t z = fso_mix64(seed + ((uint64_t)pass + 1) * FSO_GAMMA);
    const uint64_t n = (uint64_t)i * (uint64_t)B + (uint64_t)j;
    return fso_mix64(z + (n + 1) * FSO_GAMMA);
}

typedef struct {
    uint64_t pi;
    int32_t slot, j;
} fso_move;

static int fso_move_cmp(const void *a, const void *b)
{
    const uint64_t x = ((const fso_move *)a)->pi, y = ((const fso_move *)b)->pi;
    return (x > y) - (x < y);
}

static int fso_improves(int32_t cov_a, int64_t dist_a, int32_t cov_b, int64_t dist_b)
{
    if (cov_a != cov_b) return cov_a > cov_b;
    return dist_a < dist_b;
}

/* Permuted first-improvement search: mode 2 = local search (Algorithm 2),
 * mode 3 = Tabu search with improving-only acceptance (Algorithm 3), N
 * iterations from init_open (or the base ranking when NULL).  Outputs as
 * fso_tabu; the best placement is the current one after the last accepted
 * move.  Returns 0, or -1 on invalid arguments. */
int fso_perm_search(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K, int32_t R,
                    int32_t T, int32_t N, int32_t mode, uint64_t seed, const int32_t *init_open,
                    int32_t *best_open_out, int32_t *best_cov_out, int64_t *best_dist_out,
                    int32_t *best_iter_out, int32_t *passes_out,
                    int32_t *tr_out, int32_t *tr_in, int32_t *tr_moved,
                    int32_t *tr_cur_cov, int64_t *tr_cur_dist,
                    int32_t *tr_best_cov, int64_t *tr_best_dist)
{
    if (B < 1 || M < 1 || K < 1 || K > B || R < 0 || T < 0 || N < 0) return -1;
    if (mode != 2 && mode != 3) return -1;
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int32_t *S2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int32_t *tabu_until = (int32_t *)calloc((size_t)B, sizeof(int32_t));
    unsigned char *in_S = (unsigned char *)calloc((size_t)B, 1);
    fso_move *moves = (fso_move *)malloc(sizeof(fso_move) * ((size_t)K * (size_t)B + 1));

    if (init_open)
        memcpy(S, init_open, sizeof(int32_t) * (size_t)K);
    else
        fso_rank_bases(C, ldc, B, M, K, S, NULL, NULL);
    for (int32_t k = 0; k < K; ++k) in_S[S[k]] = 1;

    int32_t cur_cov, best_iter = 0;
    int64_t cur_dist;
    fso_placement_value(C, ldc, B, M, S, K, R, &cur_cov, &cur_dist);
    int32_t pass = 0, accepted_in_pass = 0, have_last = 0, stopped = 0;
    uint64_t last_pi = 0;

    for (int32_t t = 1; t <= N; ++t) {
        int32_t rec = t - 1, take = -1;
        int32_t new_cov = 0;
        int64_t new_dist = 0;
        if (!stopped) {
            /* the rest of this pass's order over the current moves */
            int32_t n = 0;
            for (int32_t k = 0; k < K; ++k)
                for (int32_t j = 0; j < B; ++j) {
                    if (in_S[j]) continue;
                    const uint64_t pi = fso_perm_priority(seed, pass, B, S[k], j);
                    if (have_last && pi <= last_pi) continue;
                    moves[n].pi = pi;
                    moves[n].slot = k;
                    moves[n].j = j;
                    ++n;
                }
            qsort(moves, (size_t)n, sizeof(fso_move), fso_move_cmp);
            for (int32_t q = 0; q < n && take < 0; ++q) {
                const int32_t i = S[moves[q].slot], j = moves[q].j;
                if (mode == 3 && !(tabu_until[i] < t && tabu_until[j] < t)) continue;
                memcpy(S2, S, sizeof(int32_t) * (size_t)K);
                S2[moves[q].slot] = j;
                int32_t c;
                int64_t d;
                fso_placement_value(C, ldc, B, M, S2, K, R, &c, &d);
                if (fso_improves(c, d, cur_cov, cur_dist)) {
                    take = q;
                    new_cov = c;
                    new_dist = d;
                }
            }
        }
        if (take >= 0) {
            const int32_t k = moves[take].slot, j = moves[take].j, i = S[k];
            S[k] = j;
            in_S[i] = 0;
            in_S[j] = 1;
            tabu_until[i] = t + T;
            tabu_until[j] = t + T;
            cur_cov = new_cov;
            cur_dist = new_dist;
            best_iter = t;
            last_pi = moves[take].pi;
            have_last = 1;
            accepted_in_pass = 1;
            if (tr_out) tr_out[rec] = i;
            if (tr_in) tr_in[rec] = j;
            if (tr_moved) tr_moved[rec] = 1;
        } else {
            if (!stopped) {
                if (accepted_in_pass) {   /* end of the order: a new pass */
                    pass += 1;
                    accepted_in_pass = 0;
                    have_last = 0;
                } else {
                    stopped = 1;          /* a whole pass without improvement */
                }
            }
            if (tr_out) tr_out[rec] = -1;
            if (tr_in) tr_in[rec] = -1;
            if (tr_moved) tr_moved[rec] = 0;
        }
        if (tr_cur_cov) tr_cur_cov[rec] = cur_cov;
        if (tr_cur_dist) tr_cur_dist[rec] = cur_dist;
        if (tr_best_cov) tr_best_cov[rec] = cur_cov;
        if (tr_best_dist) tr_best_dist[rec] = cur_dist;
    }

    unsigned char *mark = (unsigned char *)calloc((size_t)B, 1);
    for (int32_t k = 0; k < K; ++k) mark[S[k]] = 1;
    int32_t n = 0;
    for (int32_t b = 0; b < B; ++b)
        if (mark[b]) best_open_out[n++] = b;
    *best_cov_out = cur_cov;
    *best_dist_out = cur_dist;
    *best_iter_out = best_iter;
    if (passes_out) *passes_out = pass;
    free(mark);
    free(S);
    free(S2);
    free(tabu_until);
    free(in_S);
    free(moves);
    return 0;
}
