/*
 * fleetstage_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, obviously correct CPU implementation of what the fleet-staging
 * hot path computes, written from the paper
 *   J. Tassone, G. Pond, S. Choudhury, "Algorithms for Optimizing Fleet Staging
 *   of Air Ambulances", arXiv:2001.05291.
 * Only the test suite, the package smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code, header or table with the HIP
 * path; both are fed the same seeded inputs and their outputs are compared.
 *
 * Every routine states the passage it follows.  Where the paper is silent or
 * garbled, the reading taken is stated at the routine (and listed in the design
 * notes of the repository):
 *   - Earth radius r is a parameter (default 6,371,000 m); coordinates are
 *     latitude/longitude in degrees.
 *   - A mission is a round trip base -> pickup -> delivery -> same base
 *     (legs = 3); legs = 2 drops the pickup->delivery leg as Section 3 does.
 *   - Costs are rounded half-to-even to int32 metres.
 *   - The objective of Eq. 2 is read as "each mission is flown from its nearest
 *     open base"; missions whose nearest open base is farther than the range R
 *     are uncovered.  Placements are ordered by coverage (more is better), then
 *     total distance of covered missions (less is better).
 *   - The neighbourhood is all swaps (i open, j closed).  Tabu search takes the
 *     best admissible move every iteration (even a worsening one), with
 *     aspiration, ties broken by (coverage desc, distance asc, i asc, j asc);
 *     both bases of an executed move are tabu for the next T iterations.
 *
 * Parity status: every function below is pinned by tests that do not reuse its
 * code (closed forms, an independent distance formula, brute force, invariants,
 * hand-derived fixtures).  None is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FSO_DEG2RAD (3.14159265358979323846 / 180.0)

/* ------------------------------------------------------------------------ */
/* threads                                                                  */
/* ------------------------------------------------------------------------ */

void fso_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int fso_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Eq. 1 -- Haversine distance                                              */
/* ------------------------------------------------------------------------ */

/* Great-circle distance of Eq. 1 (Section 3) between (lat_a, lon_a) and
 * (lat_b, lon_b), given in degrees, on a sphere of radius r:
 *   d = 2 r asin( sqrt( sin^2((phi_a - phi_b)/2)
 *                       + cos(phi_a) cos(phi_b) sin^2((psi_a - psi_b)/2) ) ).
 * The radicand can exceed 1 by rounding near antipodes; it is clamped to 1. */
double fso_haversine(double lat_a, double lon_a, double lat_b, double lon_b, double r)
{
    double phi_a = lat_a * FSO_DEG2RAD;
    double phi_b = lat_b * FSO_DEG2RAD;
    double psi_a = lon_a * FSO_DEG2RAD;
    double psi_b = lon_b * FSO_DEG2RAD;
    double s_phi = sin((phi_a - phi_b) / 2.0);
    double s_psi = sin((psi_a - psi_b) / 2.0);
    double h = s_phi * s_phi + cos(phi_a) * cos(phi_b) * (s_psi * s_psi);
    if (h > 1.0) h = 1.0;
    if (h < 0.0) h = 0.0;
    return 2.0 * r * asin(sqrt(h));
}

/* Rounding of a distance in metres to the int32 cost unit: nearest integer,
 * ties to even (the current IEEE rounding mode, round-to-nearest-even). */
int32_t fso_round_metres(double x)
{
    return (int32_t)nearbyint(x);
}

/* ------------------------------------------------------------------------ */
/* Cost table -- Algorithm 1, the Distances fill                            */
/* ------------------------------------------------------------------------ */

/* Base-by-mission cost table.  Section 3 defines a mission as a pickup, a
 * delivery and a return to the same base; Algorithm 1 (Section 4.1) fills
 * Distances with, for every base and mission, the summed Haversine distance of
 * the base to that mission's pickup and delivery.
 *   legs = 3:  Cf[b][m] = (hav(b, p_m) + hav(p_m, d_m)) + hav(d_m, b)
 *   legs = 2:  Cf[b][m] =  hav(b, p_m) + hav(d_m, b)       (pickup->delivery
 *              leg ignored, as the Model section does)
 * bases: B x 2 (lat, lon) deg; missions: M x 4 (plat, plon, dlat, dlon) deg.
 * Cf (may be NULL) and C are row-major with row pitch ldc >= M. */
void fso_cost_table(const double *bases, int32_t B, const double *missions, int32_t M,
                    double r, int32_t legs, double *Cf, int32_t *C, int64_t ldc)
{
    int32_t b;
#pragma omp parallel for schedule(static)
    for (b = 0; b < B; ++b) {
        double blat = bases[2 * (int64_t)b], blon = bases[2 * (int64_t)b + 1];
        for (int32_t m = 0; m < M; ++m) {
            const double *ms = missions + 4 * (int64_t)m;
            double bp = fso_haversine(blat, blon, ms[0], ms[1], r);
            double db = fso_haversine(ms[2], ms[3], blat, blon, r);
            double v;
            if (legs == 3) {
                double pd = fso_haversine(ms[0], ms[1], ms[2], ms[3], r);
                v = (bp + pd) + db;
            } else {
                v = bp + db;
            }
            if (Cf) Cf[(int64_t)b * ldc + m] = v;
            C[(int64_t)b * ldc + m] = fso_round_metres(v);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Base ranking -- Algorithm 1, Top_Vals                                    */
/* ------------------------------------------------------------------------ */

/* Row sums of the Distances table: total distance of each base to every
 * mission (Section 4.1, the parallel row-sum step). */
void fso_row_sums(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int64_t *sums)
{
    for (int32_t b = 0; b < B; ++b) {
        int64_t s = 0;
        for (int32_t m = 0; m < M; ++m) s += C[(int64_t)b * ldc + m];
        sums[b] = s;
    }
}

/* Algorithm 1, Top_Vals: populate the K vehicle slots with the bases of the
 * minimum summed distance to every mission, one at a time, the smallest sum
 * first; equal sums go to the lower base id.  open_out receives the K chosen
 * ids in ascending id order; order_out (may be NULL) the same ids in the order
 * they were chosen; sums_out (may be NULL) the B row sums. */
void fso_rank_bases(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                    int32_t *open_out, int32_t *order_out, int64_t *sums_out)
{
    int64_t *sums = (int64_t *)malloc(sizeof(int64_t) * (size_t)B);
    unsigned char *taken = (unsigned char *)calloc((size_t)B, 1);
    fso_row_sums(C, ldc, B, M, sums);
    for (int32_t k = 0; k < K; ++k) {
        int32_t pick = -1;
        for (int32_t b = 0; b < B; ++b) {
            if (taken[b]) continue;
            if (pick < 0 || sums[b] < sums[pick]) pick = b;
        }
        taken[pick] = 1;
        if (order_out) order_out[k] = pick;
    }
    int32_t n = 0;
    for (int32_t b = 0; b < B; ++b)
        if (taken[b]) open_out[n++] = b;
    if (sums_out) memcpy(sums_out, sums, sizeof(int64_t) * (size_t)B);
    free(sums);
    free(taken);
}

/* ------------------------------------------------------------------------ */
/* Placement value -- Eq. 2 read as nearest open base, with range R         */
/* ------------------------------------------------------------------------ */

/* Value of placement S (K distinct base ids): every mission is flown from the
 * open base nearest to it (Algorithm 1, the per-mission assignment to the best
 * occupied base); it is covered if that cost is within R.
 *   cov  = number of covered missions,
 *   dist = sum of the nearest-base cost over covered missions (int64). */
void fso_placement_value(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                         const int32_t *S, int32_t K, int32_t R,
                         int32_t *cov_out, int64_t *dist_out)
{
    (void)B;
    int32_t cov = 0;
    int64_t dist = 0;
    for (int32_t m = 0; m < M; ++m) {
        int32_t v = INT32_MAX;
        for (int32_t k = 0; k < K; ++k) {
            int32_t c = C[(int64_t)S[k] * ldc + m];
            if (c < v) v = c;
        }
        if (v <= R) {
            cov += 1;
            dist += v;
        }
    }
    *cov_out = cov;
    *dist_out = dist;
}

/* Mission -> base assignment of placement S: the nearest open base, the lowest
 * id among equal costs, or -1 when even the nearest is beyond R. */
void fso_assign(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                const int32_t *S, int32_t K, int32_t R, int32_t *assign_out)
{
    (void)B;
    for (int32_t m = 0; m < M; ++m) {
        int32_t v = INT32_MAX, who = -1;
        for (int32_t k = 0; k < K; ++k) {
            int32_t s = S[k];
            int32_t c = C[(int64_t)s * ldc + m];
            if (c < v || (c == v && s < who)) {
                v = c;
                who = s;
            }
        }
        assign_out[m] = (v <= R) ? who : -1;
    }
}

/* ------------------------------------------------------------------------ */
/* Move evaluation -- Algorithm 3, the checks                               */
/* ------------------------------------------------------------------------ */

/* Score of every swap move: for open slot k (base i = S[k]) and closed base j,
 * the value of the placement S - i + j, i.e. the "total Haversine distance"
 * recomputed for each check in Algorithms 2 and 3, here as (coverage, distance).
 * The nearest open base of S - i + j for mission m is the smaller of C[j][m]
 * and the minimum over S without i, so that minimum (A_k) is formed first.
 * Output is K x B: cov_out[k*B + j], dist_out[k*B + j]; entries with j in S
 * are set to (-1, -1). */
void fso_move_scores(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                     const int32_t *S, int32_t K, int32_t R,
                     int32_t *cov_out, int64_t *dist_out)
{
    int32_t *A = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * (size_t)M);
    unsigned char *in_S = (unsigned char *)calloc((size_t)B, 1);
    for (int32_t k = 0; k < K; ++k) in_S[S[k]] = 1;
    for (int32_t k = 0; k < K; ++k) {
        for (int32_t m = 0; m < M; ++m) {
            int32_t v = INT32_MAX;
            for (int32_t s = 0; s < K; ++s) {
                if (s == k) continue;
                int32_t c = C[(int64_t)S[s] * ldc + m];
                if (c < v) v = c;
            }
            A[(int64_t)k * M + m] = v;
        }
    }
    int32_t j;
#pragma omp parallel for schedule(dynamic, 1)
    for (j = 0; j < B; ++j) {
        if (in_S[j]) {
            for (int32_t k = 0; k < K; ++k) {
                cov_out[(int64_t)k * B + j] = -1;
                dist_out[(int64_t)k * B + j] = -1;
            }
            continue;
        }
        const int32_t *Cj = C + (int64_t)j * ldc;
        for (int32_t k = 0; k < K; ++k) {
            const int32_t *Ak = A + (int64_t)k * M;
            int32_t cov = 0;
            int64_t dist = 0;
            for (int32_t m = 0; m < M; ++m) {
                int32_t v = Ak[m] < Cj[m] ? Ak[m] : Cj[m];
                if (v <= R) {
                    cov += 1;
                    dist += v;
                }
            }
            cov_out[(int64_t)k * B + j] = cov;
            dist_out[(int64_t)k * B + j] = dist;
        }
    }
    free(A);
    free(in_S);
}

/* (cov_a, dist_a) strictly better than (cov_b, dist_b): more coverage, then
 * less distance. */
static int fso_better(int32_t cov_a, int64_t dist_a, int32_t cov_b, int64_t dist_b)
{
    if (cov_a != cov_b) return cov_a > cov_b;
    return dist_a < dist_b;
}

/* ------------------------------------------------------------------------ */
/* Tabu search -- Algorithm 3 (and the local-search baseline of Algorithm 2) */
/* ------------------------------------------------------------------------ */

/* Tabu search over swap moves starting from the base-ranking placement
 * (Section 4.3, Algorithm 3), run for exactly N iterations.  Per iteration t:
 *   1. score every swap (the checks);
 *   2. a move (i, j) is admissible when neither i nor j is on the tabu list
 *      (tabu_until[i] < t and tabu_until[j] < t), or when its score is
 *      strictly better than the best found so far (aspiration);
 *   3. the admissible move of the best score is executed, ties to the lower
 *      (i, j); if no move is admissible the iteration makes no move;
 *   4. both bases of the executed move enter the tabu list for T iterations
 *      (tabu_until = t + T), and the best-so-far placement is replaced when
 *      the new one is strictly better.
 * mode 1 is the local-search baseline (Algorithm 2 read as steepest descent):
 * a move is admissible only if it strictly improves the current placement, and
 * the search stops at a local optimum (the remaining iterations make no move).
 *
 * init_open: K distinct base ids (NULL: base ranking, Algorithm 1).
 * best_open_out: K ids ascending.  trace arrays (each may be NULL) have N
 * entries: out/in base ids (-1 when no move), moved flag, current and best
 * (cov, dist) after the iteration.  Returns 0, or -1 on invalid arguments. */
int fso_tabu(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K, int32_t R,
             int32_t T, int32_t N, int32_t mode, const int32_t *init_open,
             int32_t *best_open_out, int32_t *best_cov_out, int64_t *best_dist_out,
             int32_t *best_iter_out,
             int32_t *tr_out, int32_t *tr_in, int32_t *tr_moved,
             int32_t *tr_cur_cov, int64_t *tr_cur_dist,
             int32_t *tr_best_cov, int64_t *tr_best_dist)
{
    if (B < 1 || M < 1 || K < 1 || K > B || R < 0 || T < 0 || N < 0) return -1;
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int32_t *bestS = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int32_t *tabu_until = (int32_t *)calloc((size_t)B, sizeof(int32_t));
    int32_t *sc = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * (size_t)B);
    int64_t *sd = (int64_t *)malloc(sizeof(int64_t) * (size_t)K * (size_t)B);
    unsigned char *in_S = (unsigned char *)calloc((size_t)B, 1);

    if (init_open) {
        memcpy(S, init_open, sizeof(int32_t) * (size_t)K);
    } else {
        fso_rank_bases(C, ldc, B, M, K, S, NULL, NULL);
    }
    for (int32_t k = 0; k < K; ++k) in_S[S[k]] = 1;

    int32_t cur_cov, best_cov, best_iter = 0;
    int64_t cur_dist, best_dist;
    fso_placement_value(C, ldc, B, M, S, K, R, &cur_cov, &cur_dist);
    best_cov = cur_cov;
    best_dist = cur_dist;
    memcpy(bestS, S, sizeof(int32_t) * (size_t)K);
    int stopped = 0;

    for (int32_t t = 1; t <= N; ++t) {
        int32_t pk = -1, pj = -1, pc = 0;
        int64_t pd = 0;
        if (!stopped && K < B) {
            fso_move_scores(C, ldc, B, M, S, K, R, sc, sd);
            for (int32_t k = 0; k < K; ++k) {
                int32_t i = S[k];
                for (int32_t j = 0; j < B; ++j) {
                    if (in_S[j]) continue;
                    int32_t c = sc[(int64_t)k * B + j];
                    int64_t d = sd[(int64_t)k * B + j];
                    int admissible;
                    if (mode == 1) {
                        admissible = fso_better(c, d, cur_cov, cur_dist);
                    } else {
                        admissible = (tabu_until[i] < t && tabu_until[j] < t) ||
                                     fso_better(c, d, best_cov, best_dist);
                    }
                    if (!admissible) continue;
                    int take = 0;
                    if (pk < 0) {
                        take = 1;
                    } else if (c != pc) {
                        take = c > pc;
                    } else if (d != pd) {
                        take = d < pd;
                    } else if (i != S[pk]) {
                        take = i < S[pk];
                    } else {
                        take = j < pj;
                    }
                    if (take) {
                        pk = k;
                        pj = j;
                        pc = c;
                        pd = d;
                    }
                }
            }
        }
        int32_t rec = t - 1;
        if (pk < 0) {
            if (mode == 1) stopped = 1;
            if (tr_out) tr_out[rec] = -1;
            if (tr_in) tr_in[rec] = -1;
            if (tr_moved) tr_moved[rec] = 0;
        } else {
            int32_t i = S[pk];
            S[pk] = pj;
            in_S[i] = 0;
            in_S[pj] = 1;
            tabu_until[i] = t + T;
            tabu_until[pj] = t + T;
            cur_cov = pc;
            cur_dist = pd;
            if (fso_better(cur_cov, cur_dist, best_cov, best_dist)) {
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

    /* result placement in ascending id order */
    unsigned char *mark = (unsigned char *)calloc((size_t)B, 1);
    for (int32_t k = 0; k < K; ++k) mark[bestS[k]] = 1;
    int32_t n = 0;
    for (int32_t b = 0; b < B; ++b)
        if (mark[b]) best_open_out[n++] = b;
    *best_cov_out = best_cov;
    *best_dist_out = best_dist;
    *best_iter_out = best_iter;

    free(mark);
    free(S);
    free(bestS);
    free(tabu_until);
    free(sc);
    free(sd);
    free(in_S);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exact optimum by enumeration (stand-in for the exact ILP solve)          */
/* ------------------------------------------------------------------------ */

static void fso_enum(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                     int32_t R, int32_t depth, int32_t start, int32_t *cur,
                     int32_t *mins /* (K+1) x M: mins of the chosen prefix */,
                     int32_t *best, int32_t *best_cov, int64_t *best_dist, int *have,
                     int64_t *count)
{
    if (depth == K) {
        const int32_t *v = mins + (int64_t)K * M;
        int32_t cov = 0;
        int64_t dist = 0;
        for (int32_t m = 0; m < M; ++m)
            if (v[m] <= R) {
                cov += 1;
                dist += v[m];
            }
        *count += 1;
        if (!*have || fso_better(cov, dist, *best_cov, *best_dist)) {
            *have = 1;
            *best_cov = cov;
            *best_dist = dist;
            memcpy(best, cur, sizeof(int32_t) * (size_t)K);
        }
        return;
    }
    for (int32_t b = start; b <= B - (K - depth); ++b) {
        cur[depth] = b;
        const int32_t *prev = mins + (int64_t)depth * M;
        int32_t *next = mins + (int64_t)(depth + 1) * M;
        const int32_t *row = C + (int64_t)b * ldc;
        for (int32_t m = 0; m < M; ++m) next[m] = row[m] < prev[m] ? row[m] : prev[m];
        fso_enum(C, ldc, B, M, K, R, depth + 1, b + 1, cur, mins, best, best_cov, best_dist,
                 have, count);
    }
}

/* The best placement over all C(B, K) subsets, in lexicographic order of the
 * sorted id tuples, keeping the first of equal values.  This plays the part of
 * the exact ILP optimum the paper obtains with an external solver (Section 5),
 * for the nearest-base, range-limited reading of Eq. 2. */
void fso_brute_optimum(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                       int32_t R, int32_t *best_open_out, int32_t *best_cov_out,
                       int64_t *best_dist_out, int64_t *n_placements_out)
{
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int32_t *mins = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K + 1) * (size_t)M);
    for (int32_t m = 0; m < M; ++m) mins[m] = INT32_MAX;
    int have = 0;
    int64_t count = 0;
    *best_cov_out = 0;
    *best_dist_out = 0;
    fso_enum(C, ldc, B, M, K, R, 0, 0, cur, mins, best_open_out, best_cov_out, best_dist_out,
             &have, &count);
    *n_placements_out = count;
    free(cur);
    free(mins);
}
