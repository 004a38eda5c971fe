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
    int k[4];            // centres per axis (x, y, z, t)
    int K;               // k[0] * k[1] * k[2] * k[3]
    float C[4];          // grid intervals E_d / k_d (fp32)
    float wd, wf, wp, cf;
    double eps;
    const float* field;  // [T][Z][Y][X]
    const float* xyz;    // [T][P][3]
    const float* attr;   // [T][P]
    int32_t* labels;     // [V + T * P]: field samples, then point samples [T][P]
    unsigned long long* acc;  // [K][kSlicAcc]
    double* cen;         // [K][6]: x, y, z, t, p, f
    float* cen32;        // [K][8]: the same rounded to fp32, then 2 unused
    long long* cnt;      // [K][2]: field and point samples of each centre
    uint32_t* counters;  // SlicCounter
};

// Labels from the seed cells, and their sums.
void launch_slic_init(const DevS& s, hipStream_t st);
// One assignment pass over both sample types, with the sums of the new labels.
void launch_slic_assign(const DevS& s, hipStream_t st);
// Centres from the sums (the sums cleared), compared with the previous ones.
// seed: 1 to write the seed centres first (before the first update).
void launch_slic_update(const DevS& s, int seed, hipStream_t st);

}  // namespace mf4d
