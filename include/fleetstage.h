/*
 * fleetstage.h -- C ABI of libfleetstage.so, the MI355X (gfx950) compute path for
 * fleet staging of air ambulances:
 *   J. Tassone, G. Pond, S. Choudhury, "Algorithms for Optimizing Fleet Staging
 *   of Air Ambulances", arXiv:2001.05291.
 *
 * The problem (Section 3): K vehicles are placed on K distinct bases out of B
 * candidates.  A mission m is a round trip base -> pickup -> delivery -> the
 * same base; its cost from base b is C[b][m] (int32 metres).  A placement S
 * serves every mission from its nearest open base (the objective of Eq. 2 read
 * as nearest-base assignment); a mission is covered when that cost is within
 * the range R.  Placements are ranked by coverage (more is better), then by
 * the total distance of covered missions (less is better).  The search is the
 * base ranking of Section 4.1 (Algorithm 1) followed by the Tabu search of
 * Section 4.3 (Algorithm 3) over swap moves (i open, j closed).
 *
 * Conventions for every call:
 *  - Ids are 0-based int32.  Bulk arrays are DEVICE pointers owned by the
 *    caller; small structs (fs_params, fs_score, fs_instance) are HOST pointers.
 *  - The cost table is row-major, one row per base, with a row pitch ldc
 *    (elements, ldc >= M); all B*ldc elements must be readable, the columns
 *    [M, ldc) are ignored.  Entries must lie in [0, INT32_MAX); INT32_MAX is
 *    reserved as "no base".  Values outside that range give unspecified
 *    search results but never an out-of-bounds access (costs never index
 *    memory).  Rows are read with 16-byte vector loads when ldc % 4 == 0 and C
 *    is 16-byte aligned, otherwise with 4-byte loads.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    stream-ordered.  Calls that return host-side results synchronise the
 *    stream before returning; the others return after enqueueing.
 *  - On a negative status nothing was written to outputs that the call had not
 *    validated first; fs_last_error() returns a message for the calling thread.
 *  - The library keeps no caller pointer after a call returns.
 *  - Scratch memory is allocated by the library per call, stream-ordered
 *    (hipMallocAsync/hipFreeAsync on the caller's stream).
 */
#ifndef FLEETSTAGE_H
#define FLEETSTAGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fs_status;
#define FS_OK 0
#define FS_PENDING 1          /* serve: result not ready yet */
#define FS_E_INVALID (-1)     /* argument validation failed */
#define FS_E_NOMEM (-2)       /* device or host allocation failed */
#define FS_E_DEVICE (-3)      /* a HIP runtime call failed */
#define FS_E_BUDGET (-4)      /* serve: request can never fit the HBM budget */
#define FS_E_NOTFOUND (-5)    /* serve: unknown instance or ticket */
#define FS_E_CLOSED (-6)      /* serve: server closed */
#define FS_E_INTERNAL (-7)    /* a device-side consistency check failed */

/* Message for the last non-OK status returned on the calling thread. */
const char *fs_last_error(void);
/* Library version string. */
const char *fs_version(void);

/* Search parameters.
 *  tenure     T >= 0: both bases of an executed move stay tabu for the next T
 *             iterations (Algorithm 3's TabuList / TabuCounter).
 *  iterations N >= 0: Tabu runs exactly N iterations; local search at most N.
 *  range_m    R in [0, INT32_MAX): a mission is covered when its nearest open
 *             base costs at most R metres.
 *  mode       0 = Tabu search (Algorithm 3, best admissible move with
 *             aspiration); 1 = local search baseline (Algorithm 2 read as
 *             steepest descent: strictly improving moves only, stop at a local
 *             optimum); 2 = the paper's permuted local search and 3 = its
 *             permuted Tabu search (Algorithms 2 and 3 with their random scan
 *             orders, Section 4.3): each pass scans the swaps in a random
 *             order drawn from `seed`, continues after the last accepted move
 *             and accepts the first one that strictly improves the current
 *             placement (mode 3 skips moves touching a tabu base); a pass
 *             without acceptance stops the search.  An iteration is one scan
 *             to the next acceptance or to the end of a pass.  The priority
 *             of swap (i out, j in) in pass p is
 *             mix64(mix64(seed + (p + 1) G) + (i B + j + 1) G), with mix64 the
 *             SplitMix64 output function and G = 0x9E3779B97F4A7C15.
 *  seed       scan orders of modes 2 and 3 (ignored by modes 0 and 1). */
typedef struct {
    int32_t tenure;
    int32_t iterations;
    int32_t range_m;
    int32_t mode;
    uint64_t seed;
} fs_params;

/* Best placement found: coverage and distance of covered missions, and the
 * iteration (1-based; 0 = the initial placement) at which it was reached. */
typedef struct {
    int32_t coverage;
    int32_t best_iter;
    int64_t distance;
} fs_score;

/* One iteration of the search (40 bytes).  out_base/in_base are -1 and moved
 * is 0 when no move was admissible.  cur_* is the current placement's value
 * after the iteration, best_* the best value so far. */
typedef struct {
    int32_t iter;
    int32_t out_base;
    int32_t in_base;
    int32_t moved;
    int32_t cur_cov;
    int32_t best_cov;
    int64_t cur_dist;
    int64_t best_dist;
} fs_trace_rec;

/* Cost table (Eq. 1; Algorithm 1, the Distances fill; Section 3 mission legs).
 *   Cf[b][m] = (hav(b, p_m) + hav(p_m, d_m)) + hav(d_m, b)   (legs = 3)
 *   Cf[b][m] =  hav(b, p_m) + hav(d_m, b)                     (legs = 2)
 *   C[b][m]  = Cf[b][m] rounded half to even to int32 metres,
 * with hav the haversine great-circle distance of Eq. 1 on a sphere of radius
 * earth_radius_m (0 selects 6,371,000 m), computed in FP64.
 *   base_latlon_deg  device, B x 2 doubles (lat, lon in degrees)
 *   mission_pd_deg   device, M x 4 doubles (pickup lat, lon, delivery lat, lon)
 *   C                device, B rows of pitch ldc (>= M) int32, written [0, M)
 *   Cf               device, same shape as C in doubles, or NULL
 * Errors: FS_E_INVALID for B < 1, M < 1, ldc < M, legs not 2 or 3, NULL
 * required pointer, negative radius; FS_E_INVALID also if a cost would not fit
 * int32 (radius > 1.1e8 m).  Enqueues and returns. */
fs_status fs_build_cost_table(const double *base_latlon_deg, int32_t B,
                              const double *mission_pd_deg, int32_t M,
                              double earth_radius_m, int32_t legs,
                              int32_t *C, int64_t ldc, double *Cf, void *stream);

/* The same table from indexed missions (Section 3: a mission joins two known
 * hospitals): hosp_latlon_deg (device, H x 2 degrees) and mission_ph
 * (device, M x 2 int32: pickup and delivery hospital ids).  Mission m's
 * coordinates are those of its two hospitals, and the result is bitwise the
 * direct form's for those coordinates (each leg is the same haversine,
 * which is symmetric bit for bit, and the legs are summed in the same
 * order), computed with B H + M haversines instead of 2 B M.
 * 1 <= H <= 16,384 (one FP64 leg per hospital is staged on chip);
 * FS_E_INVALID for ids outside [0, H) (after a check on
 * the device; nothing is written then) and for the checks of
 * fs_build_cost_table.  Synchronises the stream once (the id check). */
fs_status fs_build_cost_table_indexed(const double *base_latlon_deg, int32_t B,
                                      const double *hosp_latlon_deg, int32_t H,
                                      const int32_t *mission_ph, int32_t M,
                                      double earth_radius_m, int32_t legs, int32_t *C,
                                      int64_t ldc, double *Cf, void *stream);

/* Base ranking (Section 4.1, Algorithm 1's Top_Vals): row sums
 * S_b = sum_m C[b][m] (int64), and the K bases of smallest (S_b, b).
 *   open_out  device, K int32, the chosen ids in ascending id order
 *   order_out device, K int32, the chosen ids by rank (smallest sum first), or NULL
 *   row_sums  device, B int64, or NULL
 * Errors: FS_E_INVALID for B < 1, M < 1, K < 1, K > B, ldc < M, NULL C or
 * open_out.  Enqueues and returns. */
fs_status fs_rank_bases(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                        int32_t *open_out, int32_t *order_out, int64_t *row_sums,
                        void *stream);

/* Scores of every swap move of placement `open` (the checks of Algorithms 2
 * and 3): for slot k (base i = open[k]) and closed base j, the value of the
 * placement open - i + j.
 *   open     device, K distinct base ids (slot order is the row order of the output)
 *   cov_out  device, K x B int32; entry [k*B + j] for closed j, -1 for open j
 *   dist_out device, K x B int64; same layout
 * Errors: FS_E_INVALID for bad sizes, R out of range, K > 1024,
 * repeated or out-of-range ids in `open` (checked on the host after a copy).
 * Synchronises the stream (it reads `open` on the host). */
fs_status fs_move_scores(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                         const int32_t *open, int32_t K, int32_t range_m,
                         int32_t *cov_out, int64_t *dist_out, void *stream);

/* Tabu search (Section 4.3, Algorithm 3) from the base-ranking placement
 * (Algorithm 1) or from init_open, for exactly p->iterations iterations.
 * Per iteration t: every swap (i open, j closed) is scored; a move is
 * admissible when tabu_until[i] < t and tabu_until[j] < t, or when its score
 * is strictly better than the best so far (aspiration); the best admissible
 * move by (coverage desc, distance asc, i asc, j asc) is executed, or none
 * when no move is admissible; then tabu_until[i] = tabu_until[j] = t + T and
 * the best placement is replaced on strict improvement.  p->mode = 1 runs the
 * local-search baseline instead.
 *   init_open     device, K distinct ids, or NULL (base ranking)
 *   best_open_out device, K int32, best placement in ascending id order
 *   score_out     host, the best placement's value
 *   assign_out    device, M int32: nearest open base of the best placement
 *                 (lowest id among equal costs), -1 when beyond R; or NULL
 *   trace_out     device, p->iterations records, or NULL
 * Errors: FS_E_INVALID for bad sizes or parameters (T < 0, N < 0, R out of
 * range, mode not 0/1, K > 1024, bad init ids); FS_E_INTERNAL if the
 * refreshed value of the placement disagrees with the executed move's score.
 * Synchronises the stream before returning. */
fs_status fs_tabu_solve(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                        const fs_params *p, const int32_t *init_open,
                        int32_t *best_open_out, fs_score *score_out,
                        int32_t *assign_out, fs_trace_rec *trace_out, void *stream);

/* fs_tabu_solve for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, outputs, results and errors as fs_tabu_solve; the caller
 * still owns and passes every input and output buffer.  Every other device
 * buffer the solve uses is carved from a static device array of the library
 * (fs_noalloc_scratch_bytes(), 32 MiB), one per GPU, held until the process
 * ends; no hipMalloc, hipFree or allocating routine is called.
 *   - The stream must belong to the calling thread's current device.
 *   - The dense sweep and the rule-chosen sweep variant are used (no sorted
 *     lists, no autotuning); kernel timing is off during the call.
 *   - All calls on one GPU share its array, which keeps the last call's
 *     contents: calls that overlap on one GPU race, callers serialise them.
 * Errors: those of fs_tabu_solve; FS_E_INVALID, before anything is launched,
 * when the instance needs more workspace than the array holds (about
 * 12 bytes per mission plus a few hundred bytes per base: M up to about two
 * million at a few thousand bases).  Synchronises the stream before
 * returning. */
fs_status fs_tabu_solve_noalloc(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                                int32_t K, const fs_params *p, const int32_t *init_open,
                                int32_t *best_open_out, fs_score *score_out,
                                int32_t *assign_out, fs_trace_rec *trace_out, void *stream);
/* Size in bytes of the static device array fs_tabu_solve_noalloc works in. */
int64_t fs_noalloc_scratch_bytes(void);

/* Exact optimum of a small instance by enumeration: the stand-in for the
 * exact solver the paper's evaluation compares against (Section 5, Table 1).
 * Every K-subset of the B bases is scored (nearest open base per mission,
 * coverage within range_m, the (coverage desc, distance asc) order of
 * fs_tabu_solve); among equal values the first subset in lexicographic order
 * of ascending ids wins.  best_open_out (device, K): the optimum, ascending;
 * score_out (host): its value (best_iter 0); placements_out (host, or NULL):
 * C(B, K).  The table is staged in on-chip memory: FS_E_INVALID when
 * 8 (B + 1)(K + 1) + 4 B M exceeds 56 KiB, K > 16 or C(B, K) > 2^40, and for
 * the checks of fs_tabu_solve. */
fs_status fs_brute_optimum(const int32_t *C, int64_t ldc, int32_t B, int32_t M, int32_t K,
                           int32_t range_m, int32_t *best_open_out, fs_score *score_out,
                           int64_t *placements_out, void *stream);

/* ---------------------------------------------------------------- heterogeneous fleet
 *
 * The paper's full model (Section 3, Eq. 4-10): K_r rotary-wing and K_f
 * fixed-wing vehicles; bases are aerodromes (either type) or heliports
 * (rotary-wing only), at most one vehicle per base (Eq. 6, 7); a rotary-only
 * mission (rho = 1, Eq. 10) can be flown by a rotary-wing vehicle only.  Each
 * mission is flown from its nearest compatible occupied base; coverage within
 * range and the (coverage, distance) order are those of the homogeneous calls.
 * With no heliport, no rotary-only mission and K_f = 0 the calls below give
 * exactly what fs_move_scores / fs_tabu_solve give. */
typedef struct {
    int32_t rotary;              /* K_r >= 0 rotary-wing vehicles */
    int32_t fixed;               /* K_f >= 0 fixed-wing vehicles; K = K_r + K_f >= 1 */
    const int32_t *heliport;     /* device, B: nonzero = heliport, 0 = aerodrome */
    const int32_t *rotary_only;  /* device, M: nonzero = rotary-only mission, or NULL (none) */
} fs_fleet;

/* Score of every relocation of one vehicle (the typed checks of Section 4.3):
 * for slot k (base open[k], rotary[k] != 0 for a rotary-wing vehicle) and base
 * j, the value of the placement with that vehicle moved to j.  cov_out and
 * dist_out (device, K x B, row k = slot k) hold -1 where j is occupied or is a
 * heliport and the vehicle fixed-wing.  open and rotary are device arrays of K
 * (K distinct ids, exactly fleet->rotary rotary-wing, none fixed-wing on a
 * heliport).  FS_E_INVALID on any violation (nothing is written). */
fs_status fs_fleet_move_scores(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                               const fs_fleet *fleet, const int32_t *open,
                               const int32_t *rotary, int32_t range_m, int32_t *cov_out,
                               int64_t *dist_out, void *stream);

/* Tabu search (mode 0) or local search (mode 1; modes 2 and 3 are
 * FS_E_INVALID here) over vehicle relocations,
 * exactly as fs_tabu_solve otherwise (tabu list, aspiration, order (cov desc,
 * dist asc, out-base asc, in-base asc), N iterations).  init_open / init_rotary
 * (device, K) give the initial placement and its vehicle types, or init_open =
 * NULL for the typed base ranking (Algorithm 1 with its helipad quota): bases in
 * (row sum, id) order, a heliport taken only while fewer than K_r are,
 * rotary-wing vehicles on the chosen heliports and then on the best-ranked
 * chosen aerodromes, fixed-wing on the rest.  A vehicle keeps its type when it
 * moves.  best_open_out (device, K): best placement in ascending ids;
 * best_rotary_out (device, K): their vehicle types; assign_out (device, M, or
 * NULL): nearest compatible base of each mission of the best placement (lowest
 * id among equal costs) or -1; trace_out (device, N records, or NULL).
 * FS_E_INVALID for a fleet the bases cannot hold (fewer than K_f aerodromes,
 * or fewer than K usable bases) and the checks of fs_tabu_solve. */
fs_status fs_fleet_solve(const int32_t *C, int64_t ldc, int32_t B, int32_t M,
                         const fs_fleet *fleet, const fs_params *p, const int32_t *init_open,
                         const int32_t *init_rotary, int32_t *best_open_out,
                         int32_t *best_rotary_out, fs_score *score_out, int32_t *assign_out,
                         fs_trace_rec *trace_out, void *stream);

/* One instance of a batch (host struct; pointers are device pointers).
 *   C, ldc, B, M, K, range_m  as for fs_tabu_solve
 *   init_open      device K ids, or NULL (base ranking)
 *   best_open_out  device K int32, best placement in ascending id order
 *   assign_out     device M int32 (as in fs_tabu_solve), or NULL
 *   trace_out      device p->iterations records, or NULL
 *   seed           scan orders of modes 2 and 3 for this instance (the batch
 *                  ignores p->seed, so one batch can run a portfolio of seeds) */
typedef struct {
    const int32_t *C;
    int64_t ldc;
    int32_t B, M, K, range_m;
    const int32_t *init_open;
    int32_t *best_open_out;
    int32_t *assign_out;
    fs_trace_rec *trace_out;
    uint64_t seed;
} fs_instance;

/* Tabu search (Section 4.3, Algorithm 3) of n independent instances of
 * uneven size in one launch set: every kernel of an iteration covers all
 * instances through a tile table, so small and large instances share the GPU.
 * Tenure, iterations and mode come from p (p->range_m is ignored: each
 * instance has its own range).  Each instance's result, score and trace are
 * identical to fs_tabu_solve on that instance alone.
 *   inst        host array of n instances (each B <= 32768, K <= 1024)
 *   scores_out  host array of n scores
 * Errors: FS_E_INVALID names the first offending instance; FS_E_INTERNAL as
 * for fs_tabu_solve.  Synchronises the stream before returning. */
fs_status fs_tabu_solve_batch(const fs_instance *inst, int32_t n, const fs_params *p,
                              fs_score *scores_out, void *stream);

/* Repositioning server (continuous batching).  Section 1 motivates quick
 * repositioning of vehicles when demand changes, and the conclusion quick
 * updates of the model; the server keeps cost tables resident on the device,
 * takes requests that redraw some missions of a registered instance and
 * re-solve it (Tabu search, Section 4.3) warm-started from that instance's
 * previous best placement, and runs all admitted requests together: one
 * batched iteration at a time, admitting new requests between iterations as
 * slots and device memory free up.  A request's result depends only on its
 * instance's missions after its redraw, its warm start and its parameters, so
 * it is identical alone and in the mix.
 *
 * Requests on one instance run in submission order (each starts from the
 * previous one's result); requests on different instances run concurrently.
 * Cost tables count against hbm_budget_bytes together with the workspaces of
 * running requests; tables of idle instances are evicted least recently used
 * first and rebuilt from the kept coordinates when needed again. */
typedef struct {
    int64_t hbm_budget_bytes;  /* > 0 */
    int32_t max_slots;         /* requests solved concurrently, 1..4096 */
    int32_t device;            /* HIP device ordinal */
    double earth_radius_m;     /* 0 selects 6,371,000 m */
    int32_t legs;              /* 3 or 2, as for fs_build_cost_table */
    int32_t pad;
} fs_serve_config;

typedef struct {
    int64_t resident_bytes;    /* cost tables currently on the device */
    int64_t workspace_bytes;   /* workspaces of running requests */
    int64_t evictions;         /* tables evicted so far */
    int64_t rebuilds;          /* tables built (first use or after eviction) */
    int64_t steps;             /* batched iterations run */
    int64_t completed;         /* requests finished */
    int32_t running;           /* requests in slots now */
    int32_t queued;            /* requests waiting for a slot */
} fs_serve_stats;

typedef struct fs_server fs_server;

/* Starts a server on cfg->device with its own stream and scheduler thread.
 * Errors: FS_E_INVALID for a bad config; FS_E_DEVICE if the device cannot be
 * used. */
fs_status fs_serve_open(const fs_serve_config *cfg, fs_server **out);

/* Registers an instance: base coordinates (host, B x 2 degrees) and mission
 * coordinates (host, M x 4 degrees) are copied; K vehicles; range R.  The
 * cost table is built on first use.  Returns the instance id.
 * Errors: FS_E_INVALID (sizes, K > 1024, R), FS_E_BUDGET if the instance's
 * table plus one workspace can never fit the budget, FS_E_CLOSED. */
fs_status fs_serve_register(fs_server *sv, const double *base_latlon_deg, int32_t B,
                            const double *mission_pd_deg, int32_t M, int32_t K,
                            int32_t range_m, int64_t *instance_id);

/* Submits a repositioning request: missions mission_ids[0..n) (host) of the
 * instance get the new coordinates new_pd_deg (host, n x 4 degrees), then the
 * instance is re-solved with p->tenure, p->iterations and p->mode, which is
 * 0 or 1 (p->range_m and p->seed are ignored; modes 2 and 3 are FS_E_INVALID
 * here), warm-started from its previous best placement (base ranking
 * for its first request).  n may be 0.  Thread-safe.
 * Errors: FS_E_NOTFOUND (instance), FS_E_INVALID (ids, params), FS_E_CLOSED,
 * FS_E_DEVICE after a device failure. */
fs_status fs_serve_submit(fs_server *sv, int64_t instance_id, const int32_t *mission_ids,
                          const double *new_pd_deg, int32_t n, const fs_params *p,
                          uint64_t *ticket);

/* FS_PENDING while the request runs or waits; FS_OK with the best placement
 * (host, K ids ascending), its score and the latency from submission to
 * completion in seconds; the ticket is then released.  Thread-safe.
 * Errors: FS_E_NOTFOUND (unknown or already collected ticket), or the
 * request's own failure status. */
fs_status fs_serve_poll(fs_server *sv, uint64_t ticket, int32_t *open_out, fs_score *score_out,
                        double *latency_s);

/* Counters of the server.  Thread-safe. */
fs_status fs_serve_stats_get(fs_server *sv, fs_serve_stats *out);

/* Stops the scheduler, drops the requests still waiting or running, frees
 * every device buffer and the handle (which must not be used afterwards). */
fs_status fs_serve_close(fs_server *sv);

/* Diagnostics: device time of the search kernels, for roofline reporting.
 * While enabled (on = n > 0), every n-th launch of each kernel group carries a
 * pair of HIP events that the dispatch itself stamps at its start and end, on
 * the stream it is launched on (a dispatch with events is followed by a gap of
 * several microseconds, so sampling keeps the timed loop close to its untimed
 * pace); on = 0 disables, a negative value is FS_E_INVALID; groups are
 * "sweep" (move evaluation, including the chunk-merge kernel when the mission
 * axis is split), "refresh" (argmax, move application and the open-base
 * state of the new placement), "finalize" (the sparse sweep's block scoring
 * when it runs as a kernel of its own) and "score_refresh" (that scoring and
 * the refresh in one launch).
 * Enabling or disabling discards what was recorded.  Process-wide; not meant
 * for concurrent solves. */
fs_status fs_timing_enable(int32_t on);
/* Waits for the recorded events of `group`, returns their summed elapsed time
 * (milliseconds) and number of launches, and clears them.  FS_E_INVALID for an
 * unknown group name. */
fs_status fs_timing_read(const char *group, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* FLEETSTAGE_H */
