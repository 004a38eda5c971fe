// Internal declarations shared by the host API and the kernels of libmf4d.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf4d {

constexpr uint32_t kNoVoxel = 0xFFFFFFFFu;
constexpr int kBarWords = 64 + 32 * 8;  // grid-barrier counters (top, flag, 8 subs), one line each
// The tile work list of each round parity is split into kWorkSubs sub-lists
// (tile % kWorkSubs), each with its own counter on its own 128-byte line:
// appends to one counter from every wave serialise (~11 ns each), spread over
// 64 counters they do not.
constexpr int kWorkSubs = 64;
constexpr int kWcntStride = 32;  // words between sub-list counters
// Statistics summed by many blocks go to per-block slots (distinct addresses)
// and are folded into stat64 once, instead of one same-address atomic each.
constexpr int kSlots = 1024;
enum SlotStat : int {
    SL_PART_VISITS = 0,
    SL_MEMBERS_F = 1,
    SL_MEMBERS_P = 2,
    SL_ACTIVE = 3,  // tiles holding an admissible voxel-step (or deferred)
    SL_TESTED = 4,  // candidate tiles whose admissibility was read up front
    kSlotStats = 5
};

// Bit-packed tile layout of the field labels and admissibility.
// A tile covers 32 (x) x 8 (y) x 8 (z) x BT (t) voxel-steps.  One 32-bit word
// holds the 32 x-bits of one (y, z, t) row of the tile; inside a tile the word
// index is (t_l * 8 + z_l) * 8 + y_l, so the 64 words of one t-slice are the
// 64 lanes of a wavefront.  Tiles are ordered ((tt * NZt + tz) * NYt + ty) *
// NXt + tx.  Cells past the grid are inadmissible padding.
struct Geom {
    int X, Y, Z, T;
    int BT;                 // timesteps per tile (4, 8 or 16)
    int logBT;
    int NXt, NYt, NZt, NTt; // tiles per axis
    uint32_t NT;            // number of tiles
    uint32_t WPT;           // words per tile = 64 * BT
    uint64_t nwords;        // words in a padded bit array = NT * WPT
    uint32_t WCAP;          // capacity of one work sub-list = ceil(NT / kWorkSubs)
};

// Particle-step layout: particle-major rows of Tpad steps (Tpad = next power
// of two >= T when T <= 64, else T rounded up to a multiple of 64), flat
// index e = p * Tpad + t.  Per particle, W = max(1, Tpad / 64) 64-bit words
// hold one bit per step.
struct PGeom {
    int64_t P;
    int T;
    int Tpad;
    int W;
    int logTpad;  // log2(Tpad) when Tpad is a power of two, else -1
    int tr;       // particle steps per field step: step t lies in field step t / tr
};

// Counters kept in one small device array.
enum Counter : int {
    C_NWORK0 = 0,  // tiles on work list 0 (even rounds), summed from its sub-lists for the host
    C_NWORK1 = 1,  // tiles on work list 1 (odd rounds), likewise
    C_UNUSED2 = 2, // (free)
    C_NLIST = 3,   // coupled particle-steps on the flat list
    C_DROPPED = 4, // dropped seeds
    C_ERR = 5,     // set by the persistent kernel if a grid barrier timed out
    C_ROUNDS = 6,  // rounds completed by the persistent kernel
    C_NCAND = 7,   // candidate tiles
    C_RACT = 8,    // launched rounds: 1 if the current round has work (set by its sweep)
    C_JCHANGED = 9,  // Jacobi sweeps: the sweep added a node
    C_CHG0 = 10,   // some tile is flagged changed for round parity 0 (cleared by the sweep of parity 1)
    C_CHG1 = 11,   // likewise for parity 1
    C_NCOUNTERS = 16
};

enum Stat64 : int {
    S_TILE_VISITS = 0,
    S_PART_VISITS = 1,
    S_MEMBERS_F = 2,
    S_MEMBERS_P = 3,
    S_ACTIVE_TILES = 4,
    S_TILES_TESTED = 5,
    S_DEFERRED_READ = 6,
    S_PRIO_VISITS = 7,  // tiles swept by the priority pass of a score-ordered scheduler
    S_NSTAT = 8
};

// Condition under which a queued read-out runs: with counters null always;
// else only if the chunk of rounds queued before it reached the fixed point,
// i.e. fewer than `rounds` rounds had work (counters[C_ROUNDS]) or the work
// list of parity `par` for the next round is empty.  A closed gate makes the
// read-out a no-op, so that it can be queued before the host knows.
struct ReadGate {
    const uint32_t* counters;
    uint32_t rounds;
    int par;
};

// Every device buffer of a context, passed by value to the kernels.
struct Dev {
    Geom g;
    PGeom pg;
    const float* field;      // fp32 [T][Z][Y][X]
    uint32_t* Af;            // admissibility bits, tile layout
    uint32_t* Lf;            // label bits, tile layout
    uint8_t* active;         // NT: 0 no admissible voxel-step, 1 tested and has some,
                             // 2 deferred (labels cleared, admissibility not tested yet)
    uint32_t* dirty;         // 2 x NT: tile scheduled for round parity 0 / 1
    uint8_t* chg;            // 2 x NT: tile's members changed since its last pull
    uint32_t* work;          // [2][kWorkSubs][WCAP]: work sub-lists of round parity 0 / 1
    uint32_t* wcnt;          // [2][kWorkSubs] sub-list lengths, kWcntStride words apart
    const uint32_t* bins;    // [P][Tpad] voxel bit of each particle-step, or kNoVoxel
    const float* attr_t;     // [P][Tpad] particle values (NaN padding)
    unsigned long long* Ap;  // [P][W] admissibility bits
    unsigned long long* Lp;  // [P][W] label bits
    uint2* clist;            // coupled steps (flat index, voxel bit)
    uint32_t* pdirty;        // P bits: particle gained a step this round (to close)
    uint8_t* pflag;          // P: 1 if the particle is a candidate (its Ap / Lp are valid)
    unsigned long long* slots;  // kSlotStats x kSlots partial sums of per-grow statistics
    uint32_t* counters;      // Counter
    unsigned long long* stat64;
    uint32_t* bar;           // grid barrier arrival counter
    const float2* tsum;      // NT: (min, max) of the tile's field values (load time)
    const float2* psum;      // P: (min, max) of each particle's values (load time)
    uint32_t* cand;          // candidate tile list (tiles whose range meets the band)
    const uint8_t* tpred;    // NT or null: candidate tiles to test before the rounds
    float crit[4];
    int admit_all;           // 1: test every voxel-step; 0: only candidate tiles
    int forward_only;        // 1: membership runs along a trajectory from t to t + 1 only
    int pull_all;            // 1: the pull tests every coupled step, changed tile or not
                             // (the verification round of the score-ordered schedulers)
};

// ---- launchers (kernels.hip) ----
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void launch_reset(const Dev& d, hipStream_t s);
void launch_bin_particles(const Geom& g, const PGeom& pg, const float* xyz, const float* attr,
                          uint32_t* bins, float* attr_t, hipStream_t s);
void launch_summaries(const Geom& g, const float* field, float2* tsum, hipStream_t s);
void launch_particle_summaries(const PGeom& pg, const float* attr_t, float2* psum, hipStream_t s);
void launch_admit_field(const Dev& d, hipStream_t s);
void launch_admit_particles(const Dev& d, hipStream_t s);
void launch_seeds(const Dev& d, const int32_t* seeds, int64_t S, hipStream_t s);
// One round as three launches (sweep, pull, close/push); a round whose work
// list is empty does nothing, so rounds can be queued ahead of the host.
void launch_round(const Dev& d, uint32_t round, hipStream_t s, hipEvent_t* ev = nullptr);  // ev: 4 events or null
// Sum of the work sub-list lengths of parity `par` into counters[C_NWORK0 + par].
void launch_work_total(const Dev& d, int par, hipStream_t s);
// Rounds in one cooperative persistent launch; false if it cannot be launched.
bool launch_rounds_persistent(const Dev& d, uint32_t round0, uint32_t max_rounds, int device,
                              hipStream_t s);
void launch_read_field(const Dev& d, uint32_t* out, hipStream_t s, const ReadGate& gate = ReadGate{});
void launch_read_particles(const Dev& d, uint8_t* out, hipStream_t s, const ReadGate& gate = ReadGate{});
// Trajectory segments of the grown feature as uint8 [T][P] (Section 3.4).
void launch_particle_segments(const Dev& d, uint8_t* out, hipStream_t s);
// Fold one single-seed grow into per-seed ids: members of the canonical field
// words and of the particle labels that no earlier grow reached (seen_f: one
// bit per voxel-step, seen_p: [P][ceil(T / 64)] words) take id.  particle_ids
// may be null.
void launch_seed_ids(const Dev& d, const uint32_t* words, uint32_t* seen_f, unsigned long long* seen_p,
                     int32_t id, int32_t* field_ids, int32_t* particle_ids, hipStream_t s);
// Score-ordered schedulers.  Sort keys of the candidate tiles (order-
// preserving bits of the score when it reaches thr, else 0) and values (the
// tiles), count = tiles with a key.  Score: with logits ([T][bD][bH][bW] over
// 8^3-voxel brick-steps) the largest logit of the tile's brick-steps, else
// the tile's greatest field value.
void launch_priority_keys(const Dev& d, const float* logits, int bW, int bH, int bD, float thr, uint32_t* keys,
                          uint32_t* vals, uint32_t* count, hipStream_t s);
// The priority pass: the first *count tiles of list swept in list order by
// `waves` wavefronts (wave w takes items w, w + waves, ...), as in a round of
// parity 0 (they schedule for round 1).
void launch_priority_sweep(const Dev& d, const uint32_t* list, const uint32_t* count, int waves, hipStream_t s);
// The verification round's schedule: every tile holding an admissible
// voxel-step on the work list of parity par.
void launch_verify_schedule(const Dev& d, int par, hipStream_t s);
// One Jacobi sweep: the next labels (lf_nxt, lp_nxt: copies of the current
// ones on entry) gain every admissible node one edge away from the current
// labels; counters[C_JCHANGED] is set if any node was added.
void launch_jacobi(const Dev& d, const uint32_t* lf_cur, const unsigned long long* lp_cur, uint32_t* lf_nxt,
                   unsigned long long* lp_nxt, hipStream_t s);
// stat64[dst] (+)= sum of slot statistic `which` (assign: =), and those slots cleared.
void launch_fold_slots(const Dev& d, int which, int dst, hipStream_t s, bool assign = false);
// The per-grow statistics (particle visits, active and tested tiles) folded
// (added) in one launch.
void launch_fold_grow_slots(const Dev& d, hipStream_t s);
// End of a chunk of launched rounds, in one launch: the work total of parity
// par (as launch_work_total), with snap non-null a copy of counters[C_ROUNDS]
// and of that total into snap (the read-outs' gate), and the per-grow
// statistics folded (as launch_fold_grow_slots).
void launch_chunk_end(const Dev& d, int par, uint32_t* snap, hipStream_t s);

}  // namespace mf4d
