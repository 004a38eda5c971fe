// Device state of the batched (up to 256 queries) grower.
#pragma once

#include "mf4d_internal.h"

namespace mf4d {

enum BCounter : int {
    BC_NWORK0 = 0,
    BC_NWORK1 = 1,
    BC_NDIRTYP = 2,
    BC_NLIST = 3,
    BC_DROPPED = 4,
    BC_RACT = 5,    // the current round has work (set by its sweep)
    BC_ROUNDS = 6,  // rounds that had work (since last cleared by the host)
    BC_NCOUNTERS = 8
};

// Work sub-lists per round parity, and the words between their counters.
constexpr int kBSubs = 64;
constexpr int kBCntStride = 32;

// Float offsets inside the table buffer: sorted bounds (256 each), then the
// four prefix-mask tables of 257 x 8 words (field lo, field hi, particle lo,
// particle hi).
constexpr int kTabWords = 1024 + 4 * 257 * 8;

struct DevB {
    Geom g;  // tile geometry of the single-query binning (decodes particle bins)
    int X, Y, Z, T;
    int Tp;                  // particle steps (r per field step)
    int NXb, NYb, NZb, NTb;  // tiles of (1 << lx) x (1 << ly) x (1 << lz) x (1 << lt) voxel-steps
    int lx, ly, lz, lt;      // log2 of the tile extents, lx + ly + lz + lt = 9 (512 per tile)
    uint32_t NTB;
    int Q;
    int64_t P;
    int Tpad;
    const float* field;      // fp32 [T][Z][Y][X]
    const float* attr_t;     // fp32 [P][Tpad]
    uint32_t* vrank;         // [V] ranks of each voxel-step: rank_lo | rank_hi << 16
    uint32_t* prank;         // [P][Tpad] ranks of each particle-step, likewise
    const uint32_t* bins;    // [P][Tpad] tile-layout bit position or kNoVoxel
    uint32_t* fplanes;       // [V][8] labels = output
    uint32_t* pplanes;       // [T][P][8] labels = output
    const float* tab;        // kTabWords
    uint8_t* active;         // NTB (+8)
    uint32_t* dirty;         // 2 x NTB
    uint8_t* chg;            // 2 x NTB (+8)
    uint32_t* work;          // [2][kBSubs][WCAPB] work sub-lists of round parity 0 / 1
    uint32_t* wcnt;          // [2][kBSubs] sub-list lengths, kBCntStride words apart
    uint32_t WCAPB;          // capacity of one sub-list = ceil(NTB / kBSubs)
    uint2* clist;            // coupled steps (flat step index, canonical voxel index)
    uint32_t* pdirty;        // P bits
    uint32_t* dlist;         // P
    uint32_t* counters;      // BCounter
    unsigned long long* stat64;
    int forward_only;        // 1: membership runs along a trajectory from t to t + 1 only
};

void launch_b_prepare(const DevB& d, const int32_t* seeds, int64_t S, hipStream_t s);
// One round (sweep, pull, close); a round whose work list is empty does
// nothing, so rounds are queued ahead of the host.
void launch_b_round(const DevB& d, uint32_t round, hipStream_t s);
// Total length of the work list of parity par into counters[BC_NWORK0 + par].
void launch_b_work_total(const DevB& d, int par, hipStream_t s);
void launch_b_count(const DevB& d, hipStream_t s);

}  // namespace mf4d
