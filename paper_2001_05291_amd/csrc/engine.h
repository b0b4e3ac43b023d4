// Search engine shared by the single-instance solve, the ragged batch and the
// server: device-resident instance descriptors, tile tables, and the launches
// of one Tabu iteration over any set of instances.
#pragma once

#include "fs_internal.h"

namespace fs {

constexpr int kStripes = 8;          // copies of the G/L accumulators (one per XCD)
constexpr int kRefreshMissions = 64; // missions per refresh workgroup (one per lane)

// Everything one instance's kernels need; lives in device memory.
//
// Iteration t (1-based) of an instance works on placement S_t.  The G/L
// accumulators of S_t live in slot (t & 1) (the refresh of iteration t fills
// those of S_{t+1} while the scores of S_t are still being read).  The open
// and closed lists are single: a move changes one slot of each, which the
// refresh's first workgroup writes in place (any other workgroup of that
// refresh that reads the open list patches the same slot to the same value).
// The iteration number of an instance is the launch step minus start_step.
struct InstDesc {
    const int32_t *C;
    int64_t ldc;
    int32_t B, M, Mp, K, R, T, N, mode;
    uint64_t seed;           // permuted searches (modes 2, 3): seed of the scan orders
    // sparse sweep (one instance, homogeneous, K <= kSparseW): row groups are
    // blocks of kSparseW base ids (ngroups = blocks, nsplit = mission chunks);
    // for each block and mission, the block's bases in ascending (cost, id)
    // order, twice: the first kSparseHead ranks rank-major in lst_cost /
    // lst_id ([block][rank][Mp], read by every mission), and all kSparseW
    // ranks mission-major in mm_cost / mm_id ([block][Mp][rank], read only by
    // missions whose walk goes past the head)
    int32_t sparse;
    int32_t *lst_cost;
    unsigned char *lst_id;
    int32_t *mm_cost;
    unsigned char *mm_id;
    // packed lists (every cost below 2^26 - 1: any haversine table): each
    // entry is one 32-bit key (cost << 6 | local id) in lst_cost / mm_cost,
    // and lst_id / mm_id are unused; *wide is set by a build that met a wider
    // cost (the lists are then built again unpacked)
    int32_t *wide;
    int32_t *base_slot;      // B: closed slot (>= 0) or -1 - open slot
    int32_t *base_tabu;      // B: tabu expiry by base id (sparse sweep: loaded with the slot)
    int32_t nclosed, chunk, nsplit, ngroups;
    int32_t ncand;           // row-group candidates the refresh reduces (sparse with
                             // mission chunks: kScoreParts per base block)
    int32_t active;          // 0: every kernel skips this instance
    int32_t start_step;      // launch step at which this instance's iteration 0 ends
    int32_t *open;           // K      slot -> base id
    int32_t *closed;         // B - K  slot -> base id (at least one entry)
    int32_t *open_tabu;      // K      slot -> last iteration its base is tabu
    int32_t *closed_tabu;    // B - K  (kept beside the lists so that no kernel
                             //        has to look a base's tabu state up by id)
    int32_t *b1, *b2, *o1;   // Mp: nearest cost, second-nearest, nearest slot (low 16
                             // bits) and the mission kind (bit 16: rotary-only, whose
                             // nearest and second-nearest are over rotary slots only)
    Acc *acc[2];             // kStripes x (K + 1): G at [s][0], L_k at [s][1 + k]
    Candidate *cand;         // max(ngroups, 1): best admissible move per row group
    SolveState *st;
    int32_t *best_open;      // K (slot order)
    int32_t *best_sorted;    // K ascending
    int32_t *part_cov;       // nsplit x nclosed x (K + 2) when nsplit > 1
    int64_t *part_dist;
    fs_trace_rec *trace;     // N records or NULL
    int32_t *sc_cov;         // optional full score table, K x B
    int64_t *sc_dist;
    int64_t *sums;           // B row sums (base ranking), or NULL
    int32_t need_rank;       // 1: build the initial lists from the base ranking
    int32_t pad1;
    int32_t *best_out;       // K ascending ids (caller's buffer), or NULL
    int32_t *assign_out;     // M mission -> base ids (caller's buffer), or NULL
    // heterogeneous fleet (all zero / NULL for a homogeneous one: every vehicle
    // rotary-wing, every base an aerodrome, no rotary-only mission)
    int32_t typed;
    int32_t K_r;             // rotary-wing vehicles (the first K_r of a ranked placement)
    const int32_t *base_hel; // B: 1 = heliport (rotary-wing only), caller's buffer
    const int32_t *rho;      // M: 1 = rotary-only mission, caller's buffer, or NULL
    const int32_t *init_rot; // K: vehicle types of a given initial placement, or NULL
    int32_t *open_rot;       // K   slot -> 1 if its vehicle is rotary-wing (fixed per slot)
    int32_t *open_hel;       // K   slot -> 1 if its base is a heliport
    int32_t *closed_hel;     // B-K slot -> 1 if its base is a heliport
    int32_t *best_rot_sorted;// K   vehicle types of best_sorted
    int32_t *rank_order;     // B   typed ranking: bases in (row sum, id) order
    int32_t *best_rot_out;   // K   types of best_out (caller's buffer), or NULL
};

// One workgroup's share of the work.
struct Tile {
    int32_t inst;
    int32_t g;    // row group (sweep, score), mission tile (refresh) or base row (rank)
    int32_t sp;   // mission chunk (sweep)
    int32_t pad;
};

// Per-instance launch geometry chosen on the host.
struct InstPlan {
    int32_t nclosed, ngroups, nsplit, chunk;
    int32_t sparse = 0;      // row groups are base blocks of the sparse sweep
};

constexpr int kSparseW = 64;   // bases per block of the sparse sweep (one wave)
constexpr int kSparseHead = 4; // ranks of each sorted list also stored rank-major
constexpr int kSparseMaxK = 64;
constexpr int kScoreParts = 4;   // workgroups scoring one base block (16 rows each)
// Plan of the sparse sweep: blocks of kSparseW bases x mission chunks.
InstPlan plan_sparse(int32_t B, int32_t M, int32_t K, int target_wg);

// Engine configuration shared by all instances of one launch set.
struct EngineConfig {
    int J = 1;          // closed rows per sweep workgroup
    int U = 1;          // 16-byte loads per row in flight per thread
    bool vec4 = true;   // 16-byte row loads (all tables 16-byte aligned, ldc % 4 == 0)
    bool nt = true;     // non-temporal row loads
    bool queue = true;  // score only compacted c < b2 elements (wave-level LDS queue)
    bool wide = false;  // 1024-thread sweep workgroups (J <= 2, or in-place
                        // scoring with U = 1)
    int J_tall = 4;     // rows per workgroup of the sweep_tall tiles
    int U_tall = 1;
    int Kmax_tall = 1;  // largest K among the sweep_tall instances
    int Kmax_long = 1;  // largest K among the sweep_long instances
    // missions per refresh workgroup: kRefreshMissions (the waves split the
    // open slots of 64 missions) or kBlock (one mission per thread, all slots;
    // for small K and many missions); the refresh tiles are built to match
    int refresh_mpt = kRefreshMissions;
    // with refresh_mpt == kBlock: 1024-thread workgroups, four tiles of 64
    // missions whose waves split the open slots (large K over many missions)
    bool refresh_wide = false;
    int Kmax = 1;
    bool sparse = false;   // the sparse sweep (single homogeneous instance)
    bool sparse_packed = false;   // its lists hold packed 32-bit keys
    // the sparse sweep's block scoring and the refresh in one launch
    // (k_score_refresh; one instance with mission chunks)
    bool fuse_score = false;
    // persistent search: one workgroup per instance runs all N iterations
    // (k_solo); solo_lds is its dynamic LDS, sized for the largest instance
    bool persistent = false;
    bool solo_tab = false;     // the cost tables are staged in LDS too
    uint32_t solo_lds = 0;
    // some instance has a typed fleet: the sweep keeps the rotary-only
    // missions' common term apart (queued or scalar variant, U = 1, 256
    // threads; other launch sets never pay for it)
    bool typed = false;
};

// Device tables of a launch set.
struct EngineTables {
    const InstDesc *desc = nullptr;
    int ninst = 0;
    const Tile *sweep = nullptr;
    int nsweep = 0;
    // row groups of instances planned with EngineConfig::J_tall rows per
    // workgroup (tall instances among short ones; never split)
    const Tile *sweep_tall = nullptr;
    int nsweep_tall = 0;
    // the same for instances with long rows, swept by 1024-thread workgroups
    const Tile *sweep_long = nullptr;
    int nsweep_long = 0;
    const Tile *score = nullptr;   // row groups of instances with nsplit > 1
    int nscore = 0;
    const Tile *refresh = nullptr;
    int nrefresh = 0;
    const Tile *solo = nullptr;    // persistent search: one tile per instance, largest first
    int nsolo = 0;
    // one instance with the tiles of build_tiles (row group major, mission
    // chunk minor): the sweep, score and refresh kernels take their tile from
    // the block index instead of reading the table
    bool single = false;
};

// Geometry of one instance for a given J (rows per workgroup).
InstPlan plan_instance(int32_t B, int32_t M, int32_t K, int J, int target_wg);
// Rows per sweep workgroup from the median instance's closed rows and
// missions and the launch set's total closed rows.
int choose_rows_per_group(int32_t nclosed, int32_t M, int64_t total_rows, int32_t K);
// Dynamic LDS of a sweep workgroup of J rows for up to Kmax open slots.
size_t sweep_lds_of(int J, int Kmax);
int choose_unroll(int J);

// Workspace layout of one instance.
size_t instance_bytes(int32_t B, int32_t M, int32_t K, const InstPlan &p);
void carve_instance(InstDesc &d, char *base, int32_t B, int32_t M, int32_t K, const InstPlan &p);

// Host-side tile tables for a set of instance plans.
void build_tiles(const std::vector<InstPlan> &plans, const std::vector<int32_t> &Mp,
                 std::vector<Tile> &sweep, std::vector<Tile> &score,
                 std::vector<Tile> &refresh, int refresh_mpt = kRefreshMissions);

// Launches (stream-ordered).  `step` is the launch step: iteration
// step - start_step of every instance.
fs_status engine_reset(const EngineTables &t, int32_t maxB, int32_t Kmax, hipStream_t s);
// Base ranking of every instance with need_rank: row sums over the tiles
// (inst, row), then the initial open list (K smallest (sum, id), ascending
// ids) and closed list (the complement, ascending).
fs_status engine_rank_lists(const EngineTables &t, const Tile *row_tiles, int nrow_tiles,
                            int32_t Bmax, hipStream_t s);
// Heterogeneous fleets (typed instances only): heliport flags beside the open
// and closed lists, and the vehicle types of a given initial placement.
fs_status engine_fleet_lists(const EngineTables &t, hipStream_t s);
// State of the initial placement, then cur = best = its value.  step0 is the
// launch step at which the instances' iteration 0 ends (their start_step).
fs_status engine_init(const EngineTables &t, const EngineConfig &c, int32_t step0, hipStream_t s);
// Sparse sweep: the sorted lists and the base -> slot map (after engine_init).
// The lists are packed when every cost allows (c.sparse_packed tells the
// sweep which form was built).
fs_status engine_sparse_prepare(const EngineTables &t, EngineConfig &c, hipStream_t s);
// Scores every swap of every instance and keeps each row group's best
// admissible move.
fs_status engine_sweep(const EngineTables &t, const EngineConfig &c, int32_t step,
                       hipStream_t s);
// Global argmax and move (tabu list, best-so-far, trace), then the state of
// the new placement.
fs_status engine_refresh(const EngineTables &t, const EngineConfig &c, int32_t step,
                         hipStream_t s);
// Results of every instance: best placement sorted into best_out, the mission
// assignment into assign_out, and (score, error iteration) into device arrays.
fs_status engine_outputs(const EngineTables &t, const EngineConfig &c, fs_score *scores,
                         int32_t *errors, hipStream_t s);
// Persistent search: every remaining iteration of every instance in one
// launch, one workgroup per instance (after engine_init).
fs_status engine_persistent(const EngineTables &t, const EngineConfig &c, hipStream_t s);
// LDS of the persistent search's workgroup for one instance.
// (tab_B > 0: with the B x Mp table staged in LDS as well)
size_t solo_lds_of(int32_t Mp, int32_t K, int32_t nclosed, int32_t tab_B = 0);
constexpr int kSoloMaxMissions = 1 << 24;   // mission index and row in one queue word
constexpr int kSoloMaxKPersist = 64;        // nearest slot kept in one byte
fs_status engine_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
fs_status engine_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);

int env_int(const char *name, int dflt);

}  // namespace fs
