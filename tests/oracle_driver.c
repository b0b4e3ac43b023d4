/* Calls every exported function of the oracle on small seeded instances and
 * prints one FNV-1a digest of each call's outputs.  Test infrastructure: the
 * sanitizer test builds this file with the oracle's C sources twice, once
 * plainly and once with AddressSanitizer and UndefinedBehaviorSanitizer, and
 * requires every run to exit cleanly with identical output, also when the
 * table's row padding holds another value or another thread count runs.
 *
 * The instances cover row pitches above the mission count, K = 1 and K = B,
 * zero range, zero tenure, zero iterations, both leg counts of the cost table,
 * every search mode and the heterogeneous fleet's quota. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void fso_set_threads(int n);
double fso_haversine(double lat_a, double lon_a, double lat_b, double lon_b, double r);
int32_t fso_round_metres(double x);
void fso_cost_table(const double *bases, int32_t B, const double *missions, int32_t M,
                    double r, int32_t legs, double *Cf, int32_t *C, int64_t ldc);
void fso_row_sums(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int64_t *sums);
void fso_rank_bases(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                    int32_t *open_out, int32_t *order_out, int64_t *sums_out);
void fso_placement_value(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                         const int32_t *S, int32_t K, int32_t R,
                         int32_t *cov_out, int64_t *dist_out);
void fso_assign(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                const int32_t *S, int32_t K, int32_t R, int32_t *assign_out);
void fso_move_scores(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                     const int32_t *S, int32_t K, int32_t R,
                     int32_t *cov_out, int64_t *dist_out);
int fso_tabu(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K, int32_t R,
             int32_t T, int32_t N, int32_t mode, const int32_t *init_open,
             int32_t *best_open_out, int32_t *best_cov_out, int64_t *best_dist_out,
             int32_t *best_iter_out, int32_t *tr_out, int32_t *tr_in, int32_t *tr_moved,
             int32_t *tr_cur_cov, int64_t *tr_cur_dist, int32_t *tr_best_cov,
             int64_t *tr_best_dist);
void fso_brute_optimum(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                       int32_t R, int32_t *best_open_out, int32_t *best_cov_out,
                       int64_t *best_dist_out, int64_t *n_placements_out);
void fso_fleet_value(const int32_t *C, int64_t ldc, int32_t M, const int32_t *S,
                     const int32_t *rot, int32_t K, const int32_t *rotary_only, int32_t R,
                     int32_t *cov_out, int64_t *dist_out);
void fso_fleet_assign(const int32_t *C, int64_t ldc, int32_t M, const int32_t *S,
                      const int32_t *rot, int32_t K, const int32_t *rotary_only, int32_t R,
                      int32_t *assign_out);
void fso_fleet_move_scores(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                           const int32_t *S, const int32_t *rot, int32_t K,
                           const int32_t *heliport, const int32_t *rotary_only, int32_t R,
                           int32_t *cov_out, int64_t *dist_out);
int fso_fleet_rank(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K_r,
                   int32_t K_f, const int32_t *heliport, int32_t *open_out, int32_t *rot_out);
int fso_fleet_tabu(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K_r,
                   int32_t K_f, const int32_t *heliport, const int32_t *rotary_only, int32_t R,
                   int32_t T, int32_t N, int32_t mode, const int32_t *init_open,
                   const int32_t *init_rot, int32_t *best_open_out, int32_t *best_rot_out,
                   int32_t *best_cov_out, int64_t *best_dist_out, int32_t *best_iter_out,
                   int32_t *tr_out, int32_t *tr_in, int32_t *tr_moved, int32_t *tr_cur_cov,
                   int64_t *tr_cur_dist, int32_t *tr_best_cov, int64_t *tr_best_dist);
void fso_fleet_brute_optimum(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                             int32_t K_r, int32_t K_f, const int32_t *heliport,
                             const int32_t *rotary_only, int32_t R, int32_t *best_open_out,
                             int32_t *best_rot_out, int32_t *best_cov_out,
                             int64_t *best_dist_out, int64_t *n_placements_out);
uint64_t fso_mix64(uint64_t z);
uint64_t fso_perm_priority(uint64_t seed, int32_t pass, int32_t B, int32_t i, int32_t j);
int fso_perm_search(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K, int32_t R,
                    int32_t T, int32_t N, int32_t mode, uint64_t seed, const int32_t *init_open,
                    int32_t *best_open_out, int32_t *best_cov_out, int64_t *best_dist_out,
                    int32_t *best_iter_out, int32_t *passes_out, int32_t *tr_out,
                    int32_t *tr_in, int32_t *tr_moved, int32_t *tr_cur_cov,
                    int64_t *tr_cur_dist, int32_t *tr_best_cov, int64_t *tr_best_dist);

#define EARTH_R 6371008.8

/* ---- input generator (a 64-bit LCG; no arithmetic of the method) ---- */
static uint64_t g_state;
static uint32_t next_u32(void)
{
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(g_state >> 32);
}
static double uniform(double lo, double hi) { return lo + (hi - lo) * (next_u32() / 4294967296.0); }

static int32_t g_pad = -7;   /* fill of the row padding */

/* ---- digest ---- */
static uint64_t g_h;
static void h_bytes(const void *p, size_t n)
{
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) g_h = (g_h ^ c[i]) * 0x100000001b3ull;
}
static void h_begin(void) { g_h = 0xcbf29ce484222325ull; }
static void h_end(const char *what, int B, int M, int K)
{
    printf("%-20s B=%-3d M=%-4d K=%-3d %016llx\n", what, B, M, K, (unsigned long long)g_h);
}

static void *xmalloc(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* K distinct ids from [0, B), drawn by a partial Fisher-Yates shuffle */
static void draw_placement(int32_t B, int32_t K, int32_t *S)
{
    int32_t *ids = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)B);
    for (int32_t b = 0; b < B; ++b) ids[b] = b;
    for (int32_t k = 0; k < K; ++k) {
        const int32_t r = k + (int32_t)(next_u32() % (uint32_t)(B - k));
        const int32_t t = ids[k];
        ids[k] = ids[r];
        ids[r] = t;
        S[k] = ids[k];
    }
    free(ids);
}

static int fail(const char *what, int rc)
{
    fprintf(stderr, "%s returned %d\n", what, rc);
    return 1;
}

/* One instance: B bases, M missions in a row pitch ldc >= M, K vehicles. */
static int run_case(int32_t B, int32_t M, int64_t ldc, int32_t K, int32_t R, int32_t T,
                    int32_t N, int32_t legs, uint64_t seed)
{
    g_state = seed;
    double *bases = (double *)xmalloc(sizeof(double) * 2 * (size_t)B);
    double *missions = (double *)xmalloc(sizeof(double) * 4 * (size_t)M);
    for (int32_t b = 0; b < B; ++b) {
        bases[2 * b] = uniform(50.0, 54.0);
        bases[2 * b + 1] = uniform(-3.0, 1.0);
    }
    for (int32_t m = 0; m < M; ++m)
        for (int c = 0; c < 4; ++c) missions[4 * m + c] = uniform(c & 1 ? -3.0 : 50.0, c & 1 ? 1.0 : 54.0);
    const size_t cells = (size_t)B * (size_t)ldc;
    double *Cf = (double *)xmalloc(sizeof(double) * cells);
    int32_t *C = (int32_t *)xmalloc(sizeof(int32_t) * cells);
    /* the padding beyond M must never be read: runs with two fill values
     * have to print the same digests */
    for (size_t i = 0; i < cells; ++i) {
        Cf[i] = -1.0;
        C[i] = g_pad;
    }
    fso_cost_table(bases, B, missions, M, EARTH_R, legs, Cf, C, ldc);
    h_begin();
    for (int32_t b = 0; b < B; ++b) {
        h_bytes(Cf + (size_t)b * ldc, sizeof(double) * (size_t)M);
        h_bytes(C + (size_t)b * ldc, sizeof(int32_t) * (size_t)M);
    }
    h_end(legs == 3 ? "cost_table(3 legs)" : "cost_table(2 legs)", B, M, K);

    int64_t *sums = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)B);
    int32_t *open = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)K);
    int32_t *order = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)B);
    fso_row_sums(C, ldc, B, M, sums);
    h_begin();
    h_bytes(sums, sizeof(int64_t) * (size_t)B);
    h_end("row_sums", B, M, K);
    fso_rank_bases(C, ldc, B, M, K, open, order, sums);
    h_begin();
    h_bytes(open, sizeof(int32_t) * (size_t)K);
    h_bytes(order, sizeof(int32_t) * (size_t)K);   /* the K picks in pick order */
    h_bytes(sums, sizeof(int64_t) * (size_t)B);
    h_end("rank_bases", B, M, K);

    int32_t *S = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)K);
    draw_placement(B, K, S);
    int32_t cov = 0;
    int64_t dist = 0;
    int32_t *asg = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)M);
    fso_placement_value(C, ldc, B, M, S, K, R, &cov, &dist);
    fso_assign(C, ldc, B, M, S, K, R, asg);
    h_begin();
    h_bytes(&cov, sizeof cov);
    h_bytes(&dist, sizeof dist);
    h_bytes(asg, sizeof(int32_t) * (size_t)M);
    h_end("value+assign", B, M, K);

    int32_t *sc = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)K * (size_t)B);
    int64_t *sd = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)K * (size_t)B);
    fso_move_scores(C, ldc, B, M, S, K, R, sc, sd);
    h_begin();
    h_bytes(sc, sizeof(int32_t) * (size_t)K * (size_t)B);
    h_bytes(sd, sizeof(int64_t) * (size_t)K * (size_t)B);
    h_end("move_scores", B, M, K);

    const size_t n = N > 0 ? (size_t)N : 0;
    int32_t *tr[5];
    int64_t *tr64[2];
    for (int i = 0; i < 5; ++i) tr[i] = (int32_t *)xmalloc(sizeof(int32_t) * n);
    for (int i = 0; i < 2; ++i) tr64[i] = (int64_t *)xmalloc(sizeof(int64_t) * n);
    int32_t *best = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)K);
    int32_t it = 0, passes = 0;
    int bad = 0;
    for (int32_t mode = 0; mode < 4 && !bad; ++mode) {
        /* mode 0 and 2 from the base ranking, 1 and 3 from the drawn placement */
        const int32_t *init = (mode & 1) ? S : NULL;
        int rc;
        if (mode < 2)
            rc = fso_tabu(C, ldc, B, M, K, R, T, N, mode, init, best, &cov, &dist, &it, tr[0],
                          tr[1], tr[2], tr[3], tr64[0], tr[4], tr64[1]);
        else
            rc = fso_perm_search(C, ldc, B, M, K, R, T, N, mode, seed ^ 0x5bd1e995u, init, best,
                                 &cov, &dist, &it, &passes, tr[0], tr[1], tr[2], tr[3],
                                 tr64[0], tr[4], tr64[1]);
        if (rc != 0) {
            bad = fail("search", rc);
            break;
        }
        h_begin();
        h_bytes(best, sizeof(int32_t) * (size_t)K);
        h_bytes(&cov, sizeof cov);
        h_bytes(&dist, sizeof dist);
        h_bytes(&it, sizeof it);
        h_bytes(&passes, sizeof passes);
        for (int i = 0; i < 5; ++i) h_bytes(tr[i], sizeof(int32_t) * n);
        for (int i = 0; i < 2; ++i) h_bytes(tr64[i], sizeof(int64_t) * n);
        static const char *names[4] = {"tabu", "local_search", "perm_local", "perm_tabu"};
        h_end(names[mode], B, M, K);
    }

    /* the same searches with every trace pointer NULL */
    if (!bad) {
        int rc = fso_tabu(C, ldc, B, M, K, R, T, N, 0, NULL, best, &cov, &dist, &it, NULL, NULL,
                          NULL, NULL, NULL, NULL, NULL);
        if (rc == 0)
            rc = fso_perm_search(C, ldc, B, M, K, R, T, N, 3, seed, NULL, best, &cov, &dist,
                                 &it, &passes, NULL, NULL, NULL, NULL, NULL, NULL, NULL);
        if (rc != 0) bad = fail("search without trace", rc);
    }

    /* heterogeneous fleet: about half the vehicles rotary, a third of the
     * bases heliports (at most K_r), a quarter of the missions rotary-only */
    int32_t *heli = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)B);
    int32_t *ronly = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)M);
    int32_t *rot = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)K);
    int32_t *brot = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)K);
    const int32_t K_r = K / 2, K_f = K - K_r;
    /* at most K_r heliports, so that the bases can always hold the fleet */
    int32_t nheli = 0;
    for (int32_t b = 0; b < B; ++b) {
        heli[b] = nheli < K_r && (next_u32() % 3u) == 0;
        nheli += heli[b];
    }
    for (int32_t m = 0; m < M; ++m) ronly[m] = (next_u32() % 4u) == 0;
    if (!bad) {
        int rc = fso_fleet_rank(C, ldc, B, M, K_r, K_f, heli, open, rot);
        if (rc != 0) bad = fail("fleet_rank", rc);
    }
    if (!bad) {
        h_begin();
        h_bytes(open, sizeof(int32_t) * (size_t)K);
        h_bytes(rot, sizeof(int32_t) * (size_t)K);
        fso_fleet_value(C, ldc, M, open, rot, K, ronly, R, &cov, &dist);
        fso_fleet_assign(C, ldc, M, open, rot, K, ronly, R, asg);
        h_bytes(&cov, sizeof cov);
        h_bytes(&dist, sizeof dist);
        h_bytes(asg, sizeof(int32_t) * (size_t)M);
        fso_fleet_move_scores(C, ldc, B, M, open, rot, K, heli, ronly, R, sc, sd);
        h_bytes(sc, sizeof(int32_t) * (size_t)K * (size_t)B);
        h_bytes(sd, sizeof(int64_t) * (size_t)K * (size_t)B);
        h_end("fleet rank+scores", B, M, K);
        for (int32_t mode = 0; mode < 2 && !bad; ++mode) {
            const int rc = fso_fleet_tabu(C, ldc, B, M, K_r, K_f, heli, ronly, R, T, N, mode,
                                          mode ? open : NULL, mode ? rot : NULL, best, brot,
                                          &cov, &dist, &it, tr[0], tr[1], tr[2], tr[3], tr64[0],
                                          tr[4], tr64[1]);
            if (rc != 0) {
                bad = fail("fleet_tabu", rc);
                break;
            }
            h_begin();
            h_bytes(best, sizeof(int32_t) * (size_t)K);
            h_bytes(brot, sizeof(int32_t) * (size_t)K);
            h_bytes(&cov, sizeof cov);
            h_bytes(&dist, sizeof dist);
            h_bytes(&it, sizeof it);
            for (int i = 0; i < 5; ++i) h_bytes(tr[i], sizeof(int32_t) * n);
            for (int i = 0; i < 2; ++i) h_bytes(tr64[i], sizeof(int64_t) * n);
            h_end(mode ? "fleet_local_search" : "fleet_tabu", B, M, K);
        }
    }

    /* exhaustive optima on the small instances only */
    if (!bad && B <= 12) {
        int64_t count = 0;
        fso_brute_optimum(C, ldc, B, M, K, R, best, &cov, &dist, &count);
        h_begin();
        h_bytes(best, sizeof(int32_t) * (size_t)K);
        h_bytes(&cov, sizeof cov);
        h_bytes(&dist, sizeof dist);
        h_bytes(&count, sizeof count);
        h_end("brute_optimum", B, M, K);
        fso_fleet_brute_optimum(C, ldc, B, M, K_r, K_f, heli, ronly, R, best, brot, &cov, &dist,
                                &count);
        h_begin();
        h_bytes(best, sizeof(int32_t) * (size_t)K);
        h_bytes(brot, sizeof(int32_t) * (size_t)K);
        h_bytes(&cov, sizeof cov);
        h_bytes(&dist, sizeof dist);
        h_bytes(&count, sizeof count);
        h_end("fleet_brute_optimum", B, M, K);
    }

    free(bases);
    free(missions);
    free(Cf);
    free(C);
    free(sums);
    free(open);
    free(order);
    free(S);
    free(asg);
    free(sc);
    free(sd);
    for (int i = 0; i < 5; ++i) free(tr[i]);
    for (int i = 0; i < 2; ++i) free(tr64[i]);
    free(best);
    free(heli);
    free(ronly);
    free(rot);
    free(brot);
    return bad;
}

int main(int argc, char **argv)
{
    /* arguments: OpenMP threads, padding fill */
    fso_set_threads(argc > 1 ? atoi(argv[1]) : 2);
    if (argc > 2) g_pad = (int32_t)atoi(argv[2]);

    /* scalar helpers, including the half-way rounding cases */
    h_begin();
    static const double xs[] = {0.0, 0.5, 1.5, 2.5, 1e6 + 0.5, 1e6 + 0.49999, 3.25e6};
    for (size_t i = 0; i < sizeof xs / sizeof xs[0]; ++i) {
        const int32_t v = fso_round_metres(xs[i]);
        h_bytes(&v, sizeof v);
    }
    for (int i = 0; i < 64; ++i) {
        /* one draw per statement: the order of a call's arguments is unspecified */
        const double lat_a = uniform(-89, 89);
        const double lon_a = uniform(-179, 179);
        const double lat_b = uniform(-89, 89);
        const double lon_b = uniform(-179, 179);
        const double d = fso_haversine(lat_a, lon_a, lat_b, lon_b, EARTH_R);
        h_bytes(&d, sizeof d);
        const uint64_t z = fso_mix64((uint64_t)i * 0x9E3779B97F4A7C15ull);
        const uint64_t p = fso_perm_priority(0x1234u + (uint64_t)i, i % 5, 37, i % 7, i % 37);
        h_bytes(&z, sizeof z);
        h_bytes(&p, sizeof p);
    }
    h_end("scalars", 0, 0, 0);

    int bad = 0;
    /*         B    M    ldc  K   R        T  N   legs seed */
    bad |= run_case(9, 40, 40, 3, 400000, 2, 12, 3, 1);
    bad |= run_case(9, 37, 48, 9, 400000, 1, 5, 2, 2);      /* K = B, padded pitch */
    bad |= run_case(12, 64, 70, 1, 0, 0, 6, 3, 3);          /* K = 1, R = 0, T = 0 */
    bad |= run_case(11, 1, 3, 4, 900000, 3, 8, 3, 4);       /* one mission */
    bad |= run_case(40, 257, 260, 7, 350000, 3, 0, 3, 5);   /* N = 0 */
    bad |= run_case(64, 300, 300, 10, 300000, 4, 20, 2, 6);
    return bad;
}
