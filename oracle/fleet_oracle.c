/*
 * fleet_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * The heterogeneous-fleet model of the paper (Section 3, Eq. 2-10; the typed
 * part of Algorithm 1), as a plain CPU reference for the typed HIP path.  Same status
 * and rules as fleetstage_oracle.c: loaded only by the tests, the smoke check
 * and the benchmark's CPU baseline; shares no code with the HIP path.
 *
 * Readings of the paper followed here:
 *   - Bases are aerodromes, which can hold either vehicle type, or heliports,
 *     which hold rotary-wing vehicles only; every base holds at most one
 *     vehicle (Eq. 6, 7).  heliport[b] = 1 marks a heliport.
 *   - The fleet is K_r rotary-wing and K_f fixed-wing vehicles, each at one
 *     base (Eq. 4, 5).  A placement is K = K_r + K_f occupied bases, each with
 *     the type of its vehicle (rot[k] = 1 for rotary-wing).
 *   - A mission with rotary_only[m] = 1 (rho = 1) can be flown by a rotary-wing
 *     vehicle only (Eq. 10); any other mission by either type.  Without
 *     capacity (Section 3) a mission is flown from its nearest compatible
 *     occupied base; range and the lexicographic (coverage, distance) order
 *     are those of the homogeneous reading.
 *   - The neighbourhood is every relocation of one vehicle from its base i to
 *     an unoccupied base j that can hold it (a fixed-wing vehicle only to an
 *     aerodrome): the base-swap neighbourhood of the homogeneous case with the
 *     type constraint.  Move order, tabu rule and aspiration are unchanged.
 *   - Base ranking (Algorithm 1 with its helipad quota): bases in ascending
 *     (row sum, id) order; once K_r heliports are chosen no further heliport
 *     is taken; rotary-wing vehicles go to the chosen heliports first, then
 *     the remaining rotary-wing vehicles to the chosen aerodromes in rank
 *     order, then the fixed-wing vehicles to the rest.
 * With no heliports, no rotary-only mission and every vehicle rotary-wing the
 * model is exactly the homogeneous one (a test pins this).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Cost of mission m from the nearest compatible base of placement (S, rot)
 * with slot skip excluded (-1: none) and base add (with rotary flag add_rot)
 * included (-1: none).  INT32_MAX when no base can fly the mission. */
static int32_t fso_nearest(const int32_t *C, int64_t ldc, const int32_t *S, const int32_t *rot,
                           int32_t K, int32_t m, int32_t need_rot, int32_t skip, int32_t add,
                           int32_t add_rot)
{
    int32_t v = INT32_MAX;
    for (int32_t k = 0; k < K; ++k) {
        if (k == skip) continue;
        if (need_rot && !rot[k]) continue;
        const int32_t c = C[(int64_t)S[k] * ldc + m];
        if (c < v) v = c;
    }
    if (add >= 0 && (!need_rot || add_rot)) {
        const int32_t c = C[(int64_t)add * ldc + m];
        if (c < v) v = c;
    }
    return v;
}

/* Value of the typed placement (Eq. 2 read as nearest compatible base). */
void fso_fleet_value(const int32_t *C, int64_t ldc, int32_t M, const int32_t *S,
                     const int32_t *rot, int32_t K, const int32_t *rotary_only, int32_t R,
                     int32_t *cov_out, int64_t *dist_out)
{
    int32_t cov = 0;
    int64_t dist = 0;
    for (int32_t m = 0; m < M; ++m) {
        const int32_t v = fso_nearest(C, ldc, S, rot, K, m, rotary_only[m], -1, -1, 0);
        if (v <= R) {
            cov += 1;
            dist += v;
        }
    }
    *cov_out = cov;
    *dist_out = dist;
}

/* Mission -> base of the typed placement: the nearest compatible base, lowest
 * id among equal costs, -1 beyond R or when no base can fly it. */
void fso_fleet_assign(const int32_t *C, int64_t ldc, int32_t M, const int32_t *S,
                      const int32_t *rot, int32_t K, const int32_t *rotary_only, int32_t R,
                      int32_t *assign_out)
{
    for (int32_t m = 0; m < M; ++m) {
        int32_t v = INT32_MAX, who = -1;
        for (int32_t k = 0; k < K; ++k) {
            if (rotary_only[m] && !rot[k]) continue;
            const int32_t s = S[k];
            const int32_t c = C[(int64_t)s * ldc + m];
            if (c < v || (c == v && s < who)) {
                v = c;
                who = s;
            }
        }
        assign_out[m] = (who >= 0 && v <= R) ? who : -1;
    }
}

/* Score of every relocation: for slot k (base S[k], type rot[k]) and base j,
 * the value of the placement with that vehicle moved to j, recounted from the
 * definition.  K x B outputs; (-1, -1) where j is occupied or cannot hold the
 * vehicle (a heliport for a fixed-wing one). */
void fso_fleet_move_scores(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                           const int32_t *S, const int32_t *rot, int32_t K,
                           const int32_t *heliport, const int32_t *rotary_only, int32_t R,
                           int32_t *cov_out, int64_t *dist_out)
{
    unsigned char *occ = (unsigned char *)calloc((size_t)B, 1);
    for (int32_t k = 0; k < K; ++k) occ[S[k]] = 1;
    int32_t j;
#pragma omp parallel for schedule(dynamic, 1)
    for (j = 0; j < B; ++j) {
        for (int32_t k = 0; k < K; ++k) {
            const int64_t at = (int64_t)k * B + j;
            if (occ[j] || (heliport[j] && !rot[k])) {
                cov_out[at] = -1;
                dist_out[at] = -1;
                continue;
            }
            int32_t cov = 0;
            int64_t dist = 0;
            for (int32_t m = 0; m < M; ++m) {
                const int32_t v =
                    fso_nearest(C, ldc, S, rot, K, m, rotary_only[m], k, j, rot[k]);
                if (v <= R) {
                    cov += 1;
                    dist += v;
                }
            }
            cov_out[at] = cov;
            dist_out[at] = dist;
        }
    }
    free(occ);
}

/* Base ranking with types (Algorithm 1's helipad quota; reading in the header).
 * open_out: K base ids, rot_out: their vehicle types, in slot order (the
 * chosen heliports, then the chosen aerodromes, each group in rank order).
 * Returns 0, or -1 when the bases cannot hold the fleet (fewer than K_f
 * aerodromes, or fewer than K usable bases). */
int fso_fleet_rank(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K_r,
                   int32_t K_f, const int32_t *heliport, int32_t *open_out, int32_t *rot_out)
{
    const int32_t K = K_r + K_f;
    int64_t *sums = (int64_t *)malloc(sizeof(int64_t) * (size_t)B);
    unsigned char *taken = (unsigned char *)calloc((size_t)B, 1);
    int32_t *chosen = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
    for (int32_t b = 0; b < B; ++b) {
        int64_t s = 0;
        for (int32_t m = 0; m < M; ++m) s += C[(int64_t)b * ldc + m];
        sums[b] = s;
    }
    int32_t n = 0, n_hel = 0, rc = 0;
    while (n < K) {
        int32_t pick = -1;
        for (int32_t b = 0; b < B; ++b) {
            if (taken[b]) continue;
            if (heliport[b] && n_hel >= K_r) continue;
            if (pick < 0 || sums[b] < sums[pick]) pick = b;
        }
        if (pick < 0) {
            rc = -1;
            break;
        }
        taken[pick] = 1;
        chosen[n++] = pick;
        n_hel += heliport[pick] != 0;
    }
    if (rc == 0) {
        int32_t slot = 0;
        for (int32_t q = 0; q < K; ++q)   /* heliports: rotary-wing */
            if (heliport[chosen[q]]) {
                open_out[slot] = chosen[q];
                rot_out[slot++] = 1;
            }
        int32_t rot_left = K_r - n_hel;
        for (int32_t q = 0; q < K; ++q)   /* aerodromes: rotary first, then fixed */
            if (!heliport[chosen[q]]) {
                open_out[slot] = chosen[q];
                rot_out[slot++] = rot_left > 0 ? 1 : 0;
                if (rot_left > 0) rot_left -= 1;
            }
    }
    free(sums);
    free(taken);
    free(chosen);
    return rc;
}

static int fso_fleet_better(int32_t ca, int64_t da, int32_t cb, int64_t db)
{
    if (ca != cb) return ca > cb;
    return da < db;
}

/* Tabu search over relocations (Section 4.3 with the typed neighbourhood).
 * Same steps, admissibility, aspiration, tie order and tabu rule as fso_tabu;
 * a vehicle keeps its slot (and type) when it moves.  init_open/init_rot: K
 * bases and types in slot order, or NULL (typed base ranking).  Outputs: best
 * placement in slot order (bases and types), its value and iteration, and the
 * per-iteration trace.  Returns 0, or -1 on invalid arguments. */
int fso_fleet_tabu(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K_r,
                   int32_t K_f, const int32_t *heliport, const int32_t *rotary_only, int32_t R,
                   int32_t T, int32_t N, int32_t mode, const int32_t *init_open,
                   const int32_t *init_rot, int32_t *best_open_out, int32_t *best_rot_out,
                   int32_t *best_cov_out, int64_t *best_dist_out, int32_t *best_iter_out,
                   int32_t *tr_out, int32_t *tr_in, int32_t *tr_moved, int32_t *tr_cur_cov,
                   int64_t *tr_cur_dist, int32_t *tr_best_cov, int64_t *tr_best_dist)
{
    const int32_t K = K_r + K_f;
    if (B < 1 || M < 1 || K < 1 || K > B || K_r < 0 || K_f < 0 || R < 0 || T < 0 || N < 0)
        return -1;
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int32_t *rot = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int32_t *bestS = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int32_t *tabu_until = (int32_t *)calloc((size_t)B, sizeof(int32_t));
    int32_t *sc = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * (size_t)B);
    int64_t *sd = (int64_t *)malloc(sizeof(int64_t) * (size_t)K * (size_t)B);
    int rc = 0;
    if (init_open) {
        memcpy(S, init_open, sizeof(int32_t) * (size_t)K);
        memcpy(rot, init_rot, sizeof(int32_t) * (size_t)K);
    } else {
        rc = fso_fleet_rank(C, ldc, B, M, K_r, K_f, heliport, S, rot);
    }
    if (rc == 0) {
        int32_t cur_cov, best_cov, best_iter = 0;
        int64_t cur_dist, best_dist;
        fso_fleet_value(C, ldc, M, S, rot, K, rotary_only, R, &cur_cov, &cur_dist);
        best_cov = cur_cov;
        best_dist = cur_dist;
        memcpy(bestS, S, sizeof(int32_t) * (size_t)K);
        int stopped = 0;
        for (int32_t t = 1; t <= N; ++t) {
            int32_t pk = -1, pj = -1, pc = 0;
            int64_t pd = 0;
            if (!stopped && K < B) {
                fso_fleet_move_scores(C, ldc, B, M, S, rot, K, heliport, rotary_only, R, sc,
                                      sd);
                for (int32_t k = 0; k < K; ++k) {
                    const int32_t i = S[k];
                    for (int32_t j = 0; j < B; ++j) {
                        const int32_t c = sc[(int64_t)k * B + j];
                        const int64_t d = sd[(int64_t)k * B + j];
                        if (c < 0) continue;
                        int admissible;
                        if (mode == 1)
                            admissible = fso_fleet_better(c, d, cur_cov, cur_dist);
                        else
                            admissible = (tabu_until[i] < t && tabu_until[j] < t) ||
                                         fso_fleet_better(c, d, best_cov, best_dist);
                        if (!admissible) continue;
                        int take = 0;
                        if (pk < 0)
                            take = 1;
                        else if (c != pc)
                            take = c > pc;
                        else if (d != pd)
                            take = d < pd;
                        else if (i != S[pk])
                            take = i < S[pk];
                        else
                            take = j < pj;
                        if (take) {
                            pk = k;
                            pj = j;
                            pc = c;
                            pd = d;
                        }
                    }
                }
            }
            const int32_t rec = t - 1;
            if (pk < 0) {
                if (mode == 1) stopped = 1;
                if (tr_out) tr_out[rec] = -1;
                if (tr_in) tr_in[rec] = -1;
                if (tr_moved) tr_moved[rec] = 0;
            } else {
                const int32_t i = S[pk];
                S[pk] = pj;
                tabu_until[i] = t + T;
                tabu_until[pj] = t + T;
                cur_cov = pc;
                cur_dist = pd;
                if (fso_fleet_better(cur_cov, cur_dist, best_cov, best_dist)) {
                    best_cov = cur_cov;
                    best_dist = cur_dist;
                    best_iter = t;
                    memcpy(bestS, S, sizeof(int32_t) * (size_t)K);
                }
                if (tr_out) tr_out[rec] = i;
                if (tr_in) tr_in[rec] = pj;
                if (tr_moved) tr_moved[rec] = 1;
            }
            if (tr_cur_cov) tr_cur_cov[rec] = cur_cov;
            if (tr_cur_dist) tr_cur_dist[rec] = cur_dist;
            if (tr_best_cov) tr_best_cov[rec] = best_cov;
            if (tr_best_dist) tr_best_dist[rec] = best_dist;
        }
        memcpy(best_open_out, bestS, sizeof(int32_t) * (size_t)K);
        memcpy(best_rot_out, rot, sizeof(int32_t) * (size_t)K);
        *best_cov_out = best_cov;
        *best_dist_out = best_dist;
        *best_iter_out = best_iter;
    }
    free(S);
    free(rot);
    free(bestS);
    free(tabu_until);
    free(sc);
    free(sd);
    return rc;
}

/* Best typed placement by enumeration (tiny instances): every choice of K_r
 * rotary bases and K_f fixed-wing aerodromes, disjoint; first of equal values
 * in the order of the enumeration (rotary subsets, then fixed subsets, each in
 * lexicographic order of ascending ids). */
static void fso_fleet_enum_fixed(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                                 const int32_t *heliport, const int32_t *rotary_only, int32_t R,
                                 int32_t K_r, int32_t K_f, int32_t depth, int32_t start,
                                 int32_t *S, int32_t *rot, unsigned char *used, int32_t *best,
                                 int32_t *best_cov, int64_t *best_dist, int *have,
                                 int64_t *count)
{
    const int32_t K = K_r + K_f;
    if (depth == K_f) {
        int32_t cov;
        int64_t dist;
        fso_fleet_value(C, ldc, M, S, rot, K, rotary_only, R, &cov, &dist);
        *count += 1;
        if (!*have || fso_fleet_better(cov, dist, *best_cov, *best_dist)) {
            *have = 1;
            *best_cov = cov;
            *best_dist = dist;
            memcpy(best, S, sizeof(int32_t) * (size_t)K);
        }
        return;
    }
    for (int32_t b = start; b < B; ++b) {
        if (used[b] || heliport[b]) continue;
        S[K_r + depth] = b;
        rot[K_r + depth] = 0;
        used[b] = 1;
        fso_fleet_enum_fixed(C, ldc, B, M, heliport, rotary_only, R, K_r, K_f, depth + 1, b + 1,
                             S, rot, used, best, best_cov, best_dist, have, count);
        used[b] = 0;
    }
}

static void fso_fleet_enum_rot(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                               const int32_t *heliport, const int32_t *rotary_only, int32_t R,
                               int32_t K_r, int32_t K_f, int32_t depth, int32_t start,
                               int32_t *S, int32_t *rot, unsigned char *used, int32_t *best,
                               int32_t *best_cov, int64_t *best_dist, int *have, int64_t *count)
{
    if (depth == K_r) {
        fso_fleet_enum_fixed(C, ldc, B, M, heliport, rotary_only, R, K_r, K_f, 0, 0, S, rot,
                             used, best, best_cov, best_dist, have, count);
        return;
    }
    for (int32_t b = start; b < B; ++b) {
        S[depth] = b;
        rot[depth] = 1;
        used[b] = 1;
        fso_fleet_enum_rot(C, ldc, B, M, heliport, rotary_only, R, K_r, K_f, depth + 1, b + 1, S,
                           rot, used, best, best_cov, best_dist, have, count);
        used[b] = 0;
    }
}

void fso_fleet_brute_optimum(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                             int32_t K_r, int32_t K_f, const int32_t *heliport,
                             const int32_t *rotary_only, int32_t R, int32_t *best_open_out,
                             int32_t *best_rot_out, int32_t *best_cov_out,
                             int64_t *best_dist_out, int64_t *n_placements_out)
{
    const int32_t K = K_r + K_f;
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
    int32_t *rot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
    unsigned char *used = (unsigned char *)calloc((size_t)B, 1);
    int have = 0;
    int64_t count = 0;
    *best_cov_out = 0;
    *best_dist_out = 0;
    fso_fleet_enum_rot(C, ldc, B, M, heliport, rotary_only, R, K_r, K_f, 0, 0, S, rot, used,
                       best_open_out, best_cov_out, best_dist_out, &have, &count);
    for (int32_t k = 0; k < K; ++k) best_rot_out[k] = k < K_r ? 1 : 0;
    *n_placements_out = count;
    free(S);
    free(rot);
    free(used);
}
