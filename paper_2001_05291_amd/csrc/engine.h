// Search engine shared by the single-instance solve, the ragged batch and the
// server: device-resident instance descriptors, tile tables, and the launches
// of one Tabu iteration over any set of instances.
#pragma once

#include "fs_internal.h"

namespace fs {

constexpr int kStripes = 8;          // copies of the G/L accumulators (one per XCD)
constexpr int kRefreshMissions = 64; // missions per refresh workgroup (one per lane)

// Everything one instance's kernels need; lives in device memory.
struct InstDesc {
    const int32_t *C;
    int64_t ldc;
    int32_t B, M, Mp, K, R, T, N, mode;
    int32_t nclosed, chunk, nsplit, ngroups;
    int32_t active;          // 0: every kernel skips this instance
    int32_t pad0;
    int32_t *open;           // K      slot -> base id
    int32_t *closed;         // B - K  slot -> base id (at least one entry)
    int32_t *tabu_until;     // B
    int32_t *b1, *b2, *o1;   // Mp
    Acc *acc;                // kStripes x (K + 1): G at [s][0], L_k at [s][1 + k]
    Candidate *cand;         // max(ngroups, 1)
    SolveState *st;
    int32_t *best_open;      // K
    int32_t *part_cov;       // nsplit x nclosed x (K + 1) when nsplit > 1
    int64_t *part_dist;
    unsigned int *counter;   // workgroups of the current sweep that have scored
    fs_trace_rec *trace;     // N records or NULL
    int32_t *sc_cov;         // optional full score table, K x B
    int64_t *sc_dist;
    int64_t *sums;           // B row sums (base ranking), or NULL
    int32_t need_rank;       // 1: build open/closed from the base ranking on the device
    int32_t pad1;
    int32_t *best_out;       // K ascending ids (caller's buffer), or NULL
    int32_t *assign_out;     // M mission -> base ids (caller's buffer), or NULL
};

// One workgroup's share of the work.
struct Tile {
    int32_t inst;
    int32_t g;    // row group (sweep, score) or mission tile (refresh)
    int32_t sp;   // mission chunk (sweep)
    int32_t pad;
};

// Per-instance launch geometry chosen on the host.
struct InstPlan {
    int32_t nclosed, ngroups, nsplit, chunk;
};

// Engine configuration shared by all instances of one launch set.
struct EngineConfig {
    int J = 1;          // closed rows per sweep workgroup
    int U = 1;          // 16-byte loads per row in flight per thread
    bool vec4 = true;   // 16-byte row loads (all tables 16-byte aligned, ldc % 4 == 0)
    bool nt = true;     // non-temporal row loads
    bool fused = true;  // argmax/apply by the last scoring workgroup
    int Kmax = 1;
};

// Device tables of a launch set.
struct EngineTables {
    const InstDesc *desc = nullptr;
    int ninst = 0;
    const Tile *sweep = nullptr;
    int nsweep = 0;
    const Tile *score = nullptr;   // row groups of instances with nsplit > 1
    int nscore = 0;
    const Tile *refresh = nullptr;
    int nrefresh = 0;
};

// Geometry of one instance for a given J (rows per workgroup).
InstPlan plan_instance(int32_t B, int32_t M, int32_t K, int J, int target_wg);
int choose_rows_per_group(int32_t nclosed, int32_t K);
int choose_unroll(int J);

// Workspace layout of one instance.
size_t instance_bytes(int32_t B, int32_t M, int32_t K, const InstPlan &p, int32_t N_trace);
void carve_instance(InstDesc &d, char *base, int32_t B, int32_t M, int32_t K, const InstPlan &p);

// Host-side tile tables for a set of instance plans.
void build_tiles(const std::vector<InstPlan> &plans, const std::vector<int32_t> &Mp,
                 std::vector<Tile> &sweep, std::vector<Tile> &score,
                 std::vector<Tile> &refresh);

// Launches (stream-ordered).
fs_status engine_reset(const EngineTables &t, int32_t maxB, int32_t Kmax, hipStream_t s);
fs_status engine_refresh(const EngineTables &t, const EngineConfig &c, hipStream_t s);
fs_status engine_init_score(const EngineTables &t, const EngineConfig &c, hipStream_t s);
fs_status engine_sweep(const EngineTables &t, const EngineConfig &c, hipStream_t s);
fs_status engine_finalize(const EngineTables &t, const EngineConfig &c, hipStream_t s);
// Base ranking of every instance with need_rank: row sums over the tiles
// (inst, row), then the open list (K smallest (sum, id), ascending ids) and
// the closed list (the complement, ascending).
fs_status engine_rank_lists(const EngineTables &t, const Tile *row_tiles, int nrow_tiles,
                            int32_t Bmax, hipStream_t s);
// Results of every instance: best_open sorted into best_out, the mission
// assignment into assign_out, and (score, error) into host-visible arrays.
fs_status engine_outputs(const EngineTables &t, int32_t Kmax, fs_score *scores, int32_t *errors,
                         hipStream_t s);
fs_status engine_assign(const int32_t *C, int64_t ldc, int32_t M, const int32_t *open_sorted,
                        int32_t K, int32_t R, int32_t *out, hipStream_t s);
fs_status engine_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
fs_status engine_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);

int env_int(const char *name, int dflt);

}  // namespace fs
