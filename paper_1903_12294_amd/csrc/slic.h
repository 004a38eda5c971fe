// Internal declarations of the 4D SLIC clustering kernels (slic.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf4d {

// Accumulators of one centre: quantised sums (x, y, z, t, point value, field
// value) and the counts of field and point samples, as 64-bit integers.
enum SlicAcc : int { SA_X = 0, SA_Y, SA_Z, SA_T, SA_P, SA_F, SA_NF, SA_NP, kSlicAcc = 8 };

// Device counters of a run.
enum SlicCounter : int {
    SC_MOVED = 0,   // centres whose values changed by more than eps this update
    SC_RANGE = 1,   // a value outside |v| < 2048 was met (quantised sums could overflow)
    kSlicCounters = 4
};

struct DevS {
    int X, Y, Z, T;
    int64_t P;
    int Tp;              // particle steps (point sample tau at time tau / r)
    int k[4];            // centres per axis (x, y, z, t)
    int K;               // k[0] * k[1] * k[2] * k[3]
    float C[4];          // grid intervals E_d / k_d (fp32)
    float wd, wf, wp, cf;
    double eps;
    const float* field;  // [T][Z][Y][X]
    const float4* spos;  // [Tp * P]: point samples in visiting order, (x, y, z, t)
    const float* sattr;  // [Tp * P]: their values, same order
    int32_t* labels;     // [V + Tp * P]: field samples [T][Z][Y][X], then point samples in
                         // visiting order
    unsigned long long* acc;  // [K][kSlicAcc]
    double* cen;         // [K][6]: x, y, z, t, p, f
    float* cen32;        // [K][8]: the same rounded to fp32, then 2 unused
    long long* cnt;      // [K][2]: field and point samples of each centre
    // Per axis d and seed-grid slab i (centres with cell index i on axis d):
    // the least and greatest centre coordinate, as order-preserving keys,
    // at [(0 * 4 + d) * kmax + i] (least) and [(1 * 4 + d) * kmax + i].
    uint32_t* slab;
    // Per axis d and seed cell j: the least and greatest slab index whose
    // centres can reach a sample of cell j, at [(d * kmax + j) * 2] and + 1
    // (empty: least > greatest).
    int* reach;
    int mask_slabs;      // widest reach range searched through bit masks (0..32); wider ranges
                         // take the general loop
    int kmax;            // max(k[0..3])
    uint32_t* counters;  // SlicCounter
    unsigned long long* lsum;  // [K][kSlicAcc]: the sums of the last update (for the features)
};

// Cluster merging and feature statistics (Section 3.3).  Feature ids are
// centre ids (the lowest of each merged group).
enum FeatStat : int {
    FS_NF = 0, FS_NP, FS_MEAN_F, FS_MEAN_P, FS_STD_F, FS_STD_P,
    FS_XMIN, FS_XMAX, FS_YMIN, FS_YMAX, FS_ZMIN, FS_ZMAX, FS_TMIN, FS_TMAX, kFeatStats
};

struct DevM {
    int K;
    double eps;
    int* parent;             // [K] union-find links
    int32_t* feat;           // [K] feature of each centre (-1: no samples)
    unsigned long long* fsum;  // [K][kSlicAcc] integer sums per feature
    double* fmean;           // [K][2] mean field, point value per feature
    uint32_t* cext;          // [K][8] per centre: least x, y, z, t keys, then greatest
    double* css;             // [K][2] per centre: squared deviations from its feature's means
    uint32_t* fext;          // [K][8] per feature, the same
    double* fss;             // [K][2] per feature
    double* out;             // [K][kFeatStats]
    uint32_t* err;           // set if a union-find wait ran out (never expected)
};

// Merge the centres of the last run (labels, centres, counts, sums in s) and
// compute the features' statistics into m.out.  Errors as a HIP result.
int launch_slic_merge(const DevS& s, const DevM& m, hipStream_t st);

// Visiting order of the point samples: particle-steps sorted by the tile
// holding them (tile = voxel bit >> shift), steps in no voxel last; order[t *
// P + p] = the position of that step in the visiting order.  Their positions
// and times (spos; time t / r in field steps, r particle steps per field step)
// and values (sattr) are copied in that order from xyz [T][P][3] and attr
// [T][P] (T particle steps).  bins: [P][Tpad] voxel bits (~0u: none);
// scratch: nb + 1 + 1025 words, nb = number of tiles + 1.  Errors as a HIP
// result.
int launch_slic_order(const uint32_t* bins, const float* xyz, const float* attr, int64_t P, int Tpad,
                      int T, int r, int shift, uint32_t ntiles, uint32_t* scratch, uint32_t* order,
                      float4* spos, float* sattr, hipStream_t st);
// Point labels from visiting order back to [T][P]: out[q] = in[order[q]]
// (order as written by launch_slic_order).
void launch_slic_unsort(const int32_t* in, const uint32_t* order, uint64_t Q, int32_t* out, hipStream_t st);
// Trajectory segments (Section 3.4), in place on point labels [T][P]: the
// feature id (feat[label]) where the particle has that feature at t - 1 or
// t + 1, else -1.
void launch_slic_segments(int32_t* lab, const int32_t* feat, int T, int64_t P, hipStream_t st);
// Labels from the seed cells, and their sums.
void launch_slic_init(const DevS& s, hipStream_t st);
// One assignment pass over both sample types, with the sums of the new labels.
void launch_slic_assign(const DevS& s, hipStream_t st);
// Centres from the sums (the sums cleared), compared with the previous ones,
// and the slab bounds of the new centres.  seed: 1 to write the seed centres
// first (before the first update).
void launch_slic_update(const DevS& s, int seed, hipStream_t st);

}  // namespace mf4d
