// Internal declarations shared by the host API and the kernels of libmf4d.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf4d {

constexpr uint32_t kNoVoxel = 0xFFFFFFFFu;

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
};

// Counters kept in one small device array.
enum Counter : int {
    C_NWORK = 0,   // tiles on the current work list
    C_PEND0 = 1,   // pending coupled particle-steps, buffer 0
    C_PEND1 = 2,   // pending coupled particle-steps, buffer 1
    C_NDIRTYP = 3, // particles on the dirty list
    C_DROPPED = 4, // dropped seeds
    C_NCOUNTERS = 8
};

enum Stat64 : int {
    S_TILE_VISITS = 0,
    S_PART_VISITS = 1,
    S_MEMBERS_F = 2,
    S_MEMBERS_P = 3,
    S_ACTIVE_TILES = 4,
    S_NSTAT = 8
};

// ---- launchers (kernels.hip) ----
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void launch_bin_particles(const Geom& g, const PGeom& pg, const float* xyz, const float* attr,
                          uint32_t* bins, float* attr_t, hipStream_t s);
void launch_admit_field(const Geom& g, const float* field, float lo, float hi, uint32_t* A,
                        uint8_t* active, hipStream_t s);
void launch_count_active(const Geom& g, const uint8_t* active, unsigned long long* stat,
                         hipStream_t s);
void launch_admit_particles(const PGeom& pg, const float* attr_t, const uint32_t* bins, float lo,
                            float hi, unsigned long long* Ap, uint2* pend, uint32_t* npend,
                            hipStream_t s);
void launch_seeds(const Geom& g, const int32_t* seeds, int64_t S, const uint32_t* A, uint32_t* L,
                  const uint8_t* active, uint8_t* dirty, uint32_t* dropped, hipStream_t s);
void launch_compact_tiles(const Geom& g, uint8_t* dirty, uint32_t* work, uint32_t* nwork,
                          hipStream_t s);
void launch_mark_work(const uint32_t* work, const uint32_t* nwork, uint32_t nwork_host,
                      uint8_t* dirty, hipStream_t s);
void launch_sweep(const Geom& g, const uint32_t* A, uint32_t* L, const uint8_t* active,
                  const uint32_t* work, const uint32_t* nwork, uint32_t nwork_host,
                  uint8_t* dirty, unsigned long long* visits, hipStream_t s);
void launch_pull(const PGeom& pg, const uint2* pin, const uint32_t* nin, uint32_t nin_host,
                 uint2* pout, uint32_t* nout, const uint32_t* Lf, unsigned long long* Lp,
                 uint32_t* pdirty, uint32_t* dlist, uint32_t* ndlist, hipStream_t s);
void launch_close_push(const Geom& g, const PGeom& pg, const uint32_t* dlist,
                       const uint32_t* ndlist, uint32_t ndlist_host,
                       const unsigned long long* Ap, unsigned long long* Lp, uint32_t* pdirty,
                       const uint32_t* bins, const uint32_t* Af, uint32_t* Lf,
                       const uint8_t* active, uint8_t* dirty, unsigned long long* visits,
                       hipStream_t s);
void launch_read_field(const Geom& g, const uint32_t* L, uint32_t* out,
                       unsigned long long* members, hipStream_t s);
void launch_read_particles(const PGeom& pg, const unsigned long long* Lp, uint8_t* out,
                           unsigned long long* members, hipStream_t s);

}  // namespace mf4d
