// HIP kernels of the coupled point + field region grower, for gfx950 (wave64).
//
// Field nodes are kept as bit-packed tiles (Geom in mf4d_internal.h); the
// particle part as one bit per particle-step in 64-bit words per particle.
// Every label bit only goes 0 -> 1, so the order in which waves apply their
// updates cannot change the fixed point they reach (the least fixed point of a
// monotone operator); stale reads only delay a bit to a later round, and every
// change that another tile or particle must see schedules that work.
//
// A round has three phases: sweep the tiles on this round's work list, pull
// coupled particle-steps whose voxel joined, close the trajectories of the
// particles that gained steps and push their voxels.  Work lists, dirty flags
// and "changed" flags are double-buffered by round parity.  The phases run
// either as three launches per round or inside one cooperative persistent
// kernel separated by grid barriers.
#include <algorithm>

#include "mf4d_internal.h"

namespace mf4d {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ bool in_band(float v, float lo, float hi) { return lo <= v && v <= hi; }

// Every bit of `a` in a run (maximal block of consecutive ones) of `a` that
// holds a bit of `l` at or below it; requires l within a.  The carry of a + l
// runs from the lowest bit of l in each run to the run's top.
__device__ __forceinline__ uint32_t fill_up32(uint32_t l, uint32_t a) {
    return (((a + l) ^ a) & a) | l;
}
__device__ __forceinline__ uint64_t fill_up64(uint64_t l, uint64_t a) {
    return (((a + l) ^ a) & a) | l;
}
// Whole runs of `a` that hold a bit of `l`.
__device__ __forceinline__ uint32_t fill_runs32(uint32_t l, uint32_t a) {
    const uint32_t up = fill_up32(l, a);
    const uint32_t dn = __builtin_bitreverse32(
        fill_up32(__builtin_bitreverse32(l), __builtin_bitreverse32(a)));
    return up | dn;
}
__device__ __forceinline__ uint64_t fill_runs64(uint64_t l, uint64_t a) {
    const uint64_t up = fill_up64(l, a);
    const uint64_t dn = __builtin_bitreverse64(
        fill_up64(__builtin_bitreverse64(l), __builtin_bitreverse64(a)));
    return up | dn;
}
// Trajectory closure of a label word: whole runs, or with forward-only
// coupling the part of each run at or after its first member step.
__device__ __forceinline__ uint64_t close_word(uint64_t l, uint64_t a, int forward_only) {
    return forward_only ? fill_up64(l, a) : fill_runs64(l, a);
}

__device__ __forceinline__ uint32_t tile_of(const Geom& g, int tx, int ty, int tz, int tt) {
    return ((uint32_t)(tt * g.NZt + tz) * g.NYt + ty) * g.NXt + tx;
}

__device__ __forceinline__ uint32_t bit_index(const Geom& g, int x, int y, int z, int t) {
    const int tt = t >> g.logBT;
    const uint32_t tile = tile_of(g, x >> 5, y >> 3, z >> 3, tt);
    const uint32_t word = tile * g.WPT + (uint32_t)((((t - (tt << g.logBT)) << 3) + (z & 7)) << 3) +
                          (y & 7);
    return word * 32u + (x & 31);
}

__device__ __forceinline__ void tile_coords(const Geom& g, uint32_t tile, int& tx, int& ty, int& tz,
                                            int& tt) {
    tx = tile % g.NXt;
    tile /= g.NXt;
    ty = tile % g.NYt;
    tile /= g.NYt;
    tz = tile % g.NZt;
    tt = tile / g.NZt;
}

__device__ __forceinline__ bool test_bit(const uint32_t* a, uint32_t b) {
    return (a[b >> 5] >> (b & 31)) & 1u;
}

// Canonical voxel of a tile-layout bit position.
__device__ __forceinline__ size_t voxel_of_bit(const Geom& g, uint32_t b) {
    const uint32_t word = b >> 5;
    const uint32_t wi = word & (g.WPT - 1);
    int tx, ty, tz, tt;
    tile_coords(g, word >> (6 + g.logBT), tx, ty, tz, tt);
    const int x = tx * 32 + (b & 31), y = ty * 8 + (wi & 7), z = tz * 8 + ((wi >> 3) & 7);
    const int t = (tt << g.logBT) + (wi >> 6);
    return (((size_t)t * g.Z + z) * g.Y + y) * g.X + x;
}

// Admissibility of voxel b.  A tile that is not active holds no admissible
// voxel (its bit words are not rewritten this grow); a deferred tile has not
// been tested yet, so the field value itself is tested.
__device__ __forceinline__ bool admissible_bit(const Dev& d, uint32_t b) {
    // both loads issued together; the word is in bounds for any tile
    const uint8_t a = d.active[b >> (5 + 6 + d.g.logBT)];
    const uint32_t w = d.Af[b >> 5];
    if (a == 1) return (w >> (b & 31)) & 1u;
    if (a == 2) return in_band(d.field[voxel_of_bit(d.g, b)], d.crit[0], d.crit[1]);
    return false;
}

// Admissibility words of one (z_l, y_l) row of a tile at timestep t: one
// lane's 32 x-bits (eight 16-byte non-temporal loads when whole and aligned).
__device__ __forceinline__ uint32_t row_admissibility(const Dev& d, int tx, int y, int z, int t) {
    const Geom& g = d.g;
    if (t >= g.T || y >= g.Y || z >= g.Z) return 0u;
    const float lo = d.crit[0], hi = d.crit[1];
    const float* rp = d.field + ((size_t)(t * g.Z + z) * g.Y + y) * g.X + tx * 32;
    const int nx = min(32, g.X - tx * 32);
    uint32_t w = 0;
    if ((g.X & 3) == 0 && nx == 32) {
        typedef float v4f_ __attribute__((ext_vector_type(4)));
        v4f_ v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = __builtin_nontemporal_load(reinterpret_cast<const v4f_*>(rp) + k);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            w |= ((uint32_t)in_band(v[k].x, lo, hi) | ((uint32_t)in_band(v[k].y, lo, hi) << 1) |
                  ((uint32_t)in_band(v[k].z, lo, hi) << 2) | ((uint32_t)in_band(v[k].w, lo, hi) << 3))
                 << (4 * k);
    } else {
        for (int k = 0; k < nx; ++k) w |= (uint32_t)in_band(rp[k], lo, hi) << k;
    }
    return w;
}

// Admissibility words of one t-slice of a tile (64 rows of 32 x), computed by
// the whole wave: eight lanes read one 128-byte row with 16-byte loads, so an
// instruction covers 8 whole rows; the eight nibble-words of a row are ORed
// and handed to the lane that owns the row.  Returns the word of row `lane`
// ((z_l, y_l) = (lane >> 3, lane & 7)).  Call with the whole wave.
__device__ __forceinline__ uint32_t slice_admissibility(const Dev& d, int tx, int ty, int tz, int t) {
    const Geom& g = d.g;
    const int lane = lane_id();
    if ((g.X & 3) != 0) return row_admissibility(d, tx, ty * 8 + (lane & 7), tz * 8 + (lane >> 3), t);
    if (t >= g.T) return 0u;
    typedef float v4f_ __attribute__((ext_vector_type(4)));
    const float lo = d.crit[0], hi = d.crit[1];
    const int quad = lane & 7, grp = lane >> 3;
    const int x = tx * 32 + quad * 4;
    v4f_ v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        // row i*8 + grp holds (z_l, y_l) = (i, grp)
        const int y = ty * 8 + grp, z = tz * 8 + i;
        const float nan = __builtin_nanf("");
        v[i] = (v4f_){nan, nan, nan, nan};
        if (x < g.X && y < g.Y && z < g.Z)
            v[i] = __builtin_nontemporal_load(
                reinterpret_cast<const v4f_*>(d.field + ((size_t)(t * g.Z + z) * g.Y + y) * g.X + x));
    }
    uint32_t mine = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        uint32_t w = ((uint32_t)in_band(v[i].x, lo, hi) | ((uint32_t)in_band(v[i].y, lo, hi) << 1) |
                      ((uint32_t)in_band(v[i].z, lo, hi) << 2) | ((uint32_t)in_band(v[i].w, lo, hi) << 3))
                     << (4 * quad);
        w |= __shfl_xor(w, 1);
        w |= __shfl_xor(w, 2);
        w |= __shfl_xor(w, 4);
        const uint32_t got = __shfl(w, (lane & 7) * 8);  // row i*8 + (lane & 7)
        if ((lane >> 3) == i) mine = got;
    }
    return mine;
}

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of v over a 256-thread block; `total` gets the block sum.
// Every thread of the block must call it.
__device__ __forceinline__ uint32_t block_exclusive_scan256(uint32_t v, uint32_t* s_tmp,
                                                           uint32_t& total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_tmp[wave] = x;
    __syncthreads();
    uint32_t wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += s_tmp[w];
    total = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
    __syncthreads();
    return wbase + x - v;
}

// Exclusive prefix of a 64-bit v over a 256-thread block (four 16-bit
// counters packed in one word scan together); `total` gets the block sum.
// s_tmp: 10 words.  Every thread of the block must call it.
__device__ __forceinline__ unsigned long long block_exclusive_scan256_u64(unsigned long long v, uint32_t* s_tmp,
                                                                         unsigned long long& total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    unsigned long long x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    unsigned long long* s64 = reinterpret_cast<unsigned long long*>(s_tmp);
    if (lane == 63) s64[wave] = x;
    __syncthreads();
    unsigned long long wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += s64[w];
    total = s64[0] + s64[1] + s64[2] + s64[3];
    __syncthreads();
    return wbase + x - v;
}

// Block-wide append: each thread reserves `n` slots; one atomic per block.
__device__ __forceinline__ uint32_t block_append256(uint32_t n, uint32_t* counter, uint32_t* s_tmp) {
    uint32_t total;
    const uint32_t ex = block_exclusive_scan256(n, s_tmp, total);
    if (threadIdx.x == 0) s_tmp[4] = total ? atomicAdd(counter, total) : 0u;
    __syncthreads();
    const uint32_t base = s_tmp[4];
    __syncthreads();
    return base + ex;
}

// ---------------------------------------------------------------------------
// scheduling

// Put up to 8 tiles on the work list of round parity `par` (each once per
// round), skipping tiles with no admissible voxel-step.  Each step is issued
// for all tiles before the next (flag loads, then exchanges, then appends), so
// the round trips of the tiles overlap instead of queueing.  A flag already
// seen set needs no exchange: no one clears it during this phase.
__device__ __forceinline__ void schedule_batch(const Dev& d, const uint32_t* nb, int k, int par) {
    uint32_t* dirty = d.dirty + (size_t)par * d.g.NT;
    uint32_t cur[8];
    uint8_t act[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        act[i] = 0;
        cur[i] = 1u;
        if (i < k) {
            act[i] = d.active[nb[i]];
            cur[i] = dirty[nb[i]];
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) cur[i] = (i < k && act[i] && cur[i] == 0u) ? atomicExch(&dirty[nb[i]], 1u) : 1u;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (cur[i] == 0u) {
            const uint32_t j = (uint32_t)(par * kWorkSubs) + (nb[i] & (kWorkSubs - 1));
            const uint32_t slot = atomicAdd(&d.wcnt[j * kWcntStride], 1u);
            d.work[(size_t)j * d.g.WCAP + slot] = nb[i];
        }
    }
}

// As schedule_batch, for a sweep's few neighbours: the flag exchange is
// issued with the activity loads (two round trips instead of three).  A flag
// set on a tile with no admissible voxel-step is never read: such a tile is
// never listed.
__device__ __forceinline__ void schedule_batch_direct(const Dev& d, const uint32_t* nb, int k, int par) {
    uint32_t* dirty = d.dirty + (size_t)par * d.g.NT;
    uint32_t cur[8];
    uint8_t act[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        act[i] = 0;
        cur[i] = 1u;
        if (i < k) {
            act[i] = d.active[nb[i]];
            cur[i] = atomicExch(&dirty[nb[i]], 1u);
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (i < k && act[i] && cur[i] == 0u) {
            const uint32_t j = (uint32_t)(par * kWorkSubs) + (nb[i] & (kWorkSubs - 1));
            const uint32_t slot = atomicAdd(&d.wcnt[j * kWcntStride], 1u);
            d.work[(size_t)j * d.g.WCAP + slot] = nb[i];
        }
    }
}

// As schedule_batch for up to N tiles (nb[i] = ~0u: none; all their flag
// loads, then exchanges, then appends issued together; fixed indices only, so
// that the arrays stay in registers).
template <int N>
__device__ __forceinline__ void schedule_batch_n(const Dev& d, const uint32_t* nb, int par) {
    uint32_t* dirty = d.dirty + (size_t)par * d.g.NT;
    uint32_t cur[N];
    uint8_t act[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        act[i] = 0;
        cur[i] = 1u;
        if (nb[i] != ~0u) {
            act[i] = d.active[nb[i]];
            cur[i] = dirty[nb[i]];
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) cur[i] = (nb[i] != ~0u && act[i] && cur[i] == 0u) ? atomicExch(&dirty[nb[i]], 1u) : 1u;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (cur[i] == 0u) {
            const uint32_t j = (uint32_t)(par * kWorkSubs) + (nb[i] & (kWorkSubs - 1));
            const uint32_t slot = atomicAdd(&d.wcnt[j * kWcntStride], 1u);
            d.work[(size_t)j * d.g.WCAP + slot] = nb[i];
        }
    }
}

// Voxel bits set from outside a tile sweep (seeds, particle pushes), before
// round parity `par`: each owning tile is flagged changed (its coupled steps
// must be pulled) and scheduled.  Its sweep sees the flag and schedules every
// tile across a face that holds members, since it cannot tell the bits set
// here from older ones.  Up to 4 voxels (b = kNoVoxel: none), one round trip
// per step for all of them.
__device__ void mark_voxels(const Dev& d, const uint32_t* b, int par) {
    const Geom& g = d.g;
    uint32_t nb[8];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (b[i] == kNoVoxel) continue;
        const uint32_t tile = b[i] >> (5 + 6 + g.logBT);
        bool dup = false;
        for (int j = 0; j < k; ++j) dup |= nb[j] == tile;
        if (dup) continue;
        d.chg[par * g.NT + tile] = 1;
        d.counters[C_CHG0 + par] = 1u;
        nb[k++] = tile;
    }
    schedule_batch(d, nb, k, par);
}

__device__ __forceinline__ void mark_voxel(const Dev& d, uint32_t b, int par) {
    const uint32_t v[4] = {b, kNoVoxel, kNoVoxel, kNoVoxel};
    mark_voxels(d, v, par);
}

// mark_voxels for up to N voxels (kNoVoxel: none); a tile already named by an
// earlier voxel of the lane is marked once.
template <int N>
__device__ void mark_voxels_n(const Dev& d, const uint32_t* b, int par) {
    const Geom& g = d.g;
    uint32_t tl[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        tl[i] = b[i] != kNoVoxel ? b[i] >> (5 + 6 + g.logBT) : ~0u;
#pragma unroll
        for (int j = 0; j < i; ++j)
            if (tl[j] == tl[i]) tl[i] = ~0u;
        if (tl[i] != ~0u) {
            d.chg[par * g.NT + tl[i]] = 1;
            d.counters[C_CHG0 + par] = 1u;
        }
    }
    schedule_batch_n<N>(d, tl, par);
}

// ---------------------------------------------------------------------------
// the three phases of a round

// Sweep one tile to a local fixed point with one wavefront.  Lane = (z_l, y_l);
// each lane holds the BT words of its (y, z) column over the tile's timesteps
// in registers.  Per iteration: one Jacobi step in y and z (lane shuffles),
// complete fills along x inside each word, and complete forward / backward
// passes along t.  Neighbour-tile words enter as fixed halos; when a face of
// this tile gains bits, the tile across that face is scheduled for the next
// round.  Every lane of the wave must call it.
template <int BT>
__device__ void sweep_tile(const Dev& d, uint32_t tile, int par) {
    const Geom& g = d.g;
    const int lane = lane_id();
    const int yl = lane & 7, zl = lane >> 3;
    const uint32_t sy = g.NXt, sz = g.NXt * g.NYt, st = sz * g.NZt;
    int tx, ty, tz, tt;
    tile_coords(g, tile, tx, ty, tz, tt);
    if (lane == 0) d.dirty[par * g.NT + tile] = 0u;
    uint32_t* Ab = d.Af + (size_t)tile * (64 * BT);
    uint32_t* Lb = d.Lf + (size_t)tile * (64 * BT);
    uint32_t a[BT], l[BT], l0[BT], xin[BT], yh[BT], zh[BT];
    // Every load of the visit is issued at once (one round trip): the activity
    // of the tile and its neighbours, its admissibility and label words, and
    // the halo words of every neighbour inside the grid.  Halos of inactive
    // neighbours (stale labels, zero by definition) are masked afterwards; a
    // neighbour outside the grid reads this tile's own words, masked too.
    const bool hxm = tx > 0, hxp = tx + 1 < g.NXt;
    const bool hym = yl == 0 && ty > 0, hyp = yl == 7 && ty + 1 < g.NYt;
    const bool hzm = zl == 0 && tz > 0, hzp = zl == 7 && tz + 1 < g.NZt;
    const bool htm = tt > 0, htp = tt + 1 < g.NTt;
    const size_t w = 64 * BT;
    const uint32_t* Lxm = hxm ? Lb - w : Lb;
    const uint32_t* Lxp = hxp ? Lb + w : Lb;
    const uint32_t* Ly = hym ? Lb - (size_t)sy * w : (hyp ? Lb + (size_t)sy * w : Lb);
    const int yoff = hym ? 7 : (hyp ? -7 : 0);
    const uint32_t* Lz = hzm ? Lb - (size_t)sz * w : (hzp ? Lb + (size_t)sz * w : Lb);
    const int zoff = hzm ? 56 : (hzp ? -56 : 0);
    const uint32_t* Ltm = htm ? Lb - (size_t)st * w : Lb;
    const uint32_t* Ltp = htp ? Lb + (size_t)st * w : Lb;
    const uint8_t act = d.active[tile];
    // set before this sweep only by pushes or seeds (the sweep that sets it
    // for its own changes comes later; the previous round cleared it)
    const bool pushed = d.chg[par * g.NT + tile] != 0;
    const uint8_t axm = hxm ? d.active[tile - 1] : 0, axp = hxp ? d.active[tile + 1] : 0;
    const uint8_t ay = hym ? d.active[tile - sy] : (hyp ? d.active[tile + sy] : 0);
    const uint8_t az = hzm ? d.active[tile - sz] : (hzp ? d.active[tile + sz] : 0);
    const uint8_t atm = htm ? d.active[tile - st] : 0, atp = htp ? d.active[tile + st] : 0;
    uint32_t xm[BT], xp[BT];
#pragma unroll
    for (int t = 0; t < BT; ++t) {
        a[t] = Ab[t * 64 + lane];
        l[t] = Lb[t * 64 + lane];
        xm[t] = Lxm[t * 64 + lane];
        xp[t] = Lxp[t * 64 + lane];
        yh[t] = Ly[t * 64 + lane + yoff];
        zh[t] = Lz[t * 64 + lane + zoff];
    }
    uint32_t tm = Ltm[(BT - 1) * 64 + lane];
    uint32_t tp = Ltp[lane];
#pragma unroll
    for (int t = 0; t < BT; ++t) {
        xin[t] = (axm ? (xm[t] >> 31) : 0u) | (axp ? (xp[t] << 31) : 0u);
        yh[t] = ay ? yh[t] : 0u;
        zh[t] = az ? zh[t] : 0u;
        l0[t] = l[t];
    }
    tm = atm ? tm : 0u;
    tp = atp ? tp : 0u;
    if (act == 2) {
        // deferred tile: test its admissibility now
        uint32_t any = 0;
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            a[t] = slice_admissibility(d, tx, ty, tz, (tt << g.logBT) + t);
            Ab[t * 64 + lane] = a[t];
            any |= a[t];
        }
        const bool has = __ballot(any != 0) != 0;
        if (lane == 0) {
            d.active[tile] = has ? 1 : 0;
            atomicAdd(&d.stat64[S_DEFERRED_READ], 1ull);
        }
    }
    // Byte addresses of the lanes holding this lane's in-tile y / z
    // neighbours.  An edge lane names itself: its own word is in the union
    // anyway, and the halo word brings the neighbour tile's row.
    const int iym = (yl > 0 ? lane - 1 : lane) << 2, iyp = (yl < 7 ? lane + 1 : lane) << 2;
    const int izm = (zl > 0 ? lane - 8 : lane) << 2, izp = (zl < 7 ? lane + 8 : lane) << 2;
    while (true) {
        uint32_t s[BT];
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            // one Jacobi step along y and z (lane permutes; halos for edge
            // lanes).  Measured faster than complete y/z line fills: those
            // chain 12 dependent shuffles per word.
            const int v = (int)l[t];
            const uint32_t ym = (uint32_t)__builtin_amdgcn_ds_bpermute(iym, v);
            const uint32_t yp = (uint32_t)__builtin_amdgcn_ds_bpermute(iyp, v);
            const uint32_t zm = (uint32_t)__builtin_amdgcn_ds_bpermute(izm, v);
            const uint32_t zp = (uint32_t)__builtin_amdgcn_ds_bpermute(izp, v);
            s[t] = (l[t] | xin[t] | yh[t] | zh[t] | ym | yp | zm | zp) & a[t];
        }
        // forward along t; each slice's spatial inputs and what reaches it
        // from the slice before are completed along x (runs) in one fill
        s[0] = fill_runs32(s[0] | (tm & a[0]), a[0]);
#pragma unroll
        for (int t = 1; t < BT; ++t) s[t] = fill_runs32(s[t] | (s[t - 1] & a[t]), a[t]);
        s[BT - 1] |= fill_runs32(tp & a[BT - 1], a[BT - 1]);
#pragma unroll
        for (int t = BT - 2; t >= 0; --t) s[t] |= fill_runs32(s[t + 1] & a[t], a[t]);
        uint32_t diff = 0;
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            diff |= s[t] ^ l[t];
            l[t] = s[t];
        }
        if (__ballot(diff != 0) == 0) break;
    }
    // face bits that may be new to the tile across: those this sweep set, and
    // after pushes every member (the pushed bits are not known apart)
    // A tile is swept by one wave per phase and nothing else writes its
    // words meanwhile (pushes and seeds come in other phases): a plain store.
    uint32_t any = 0, fany = 0, fx0 = 0, fx1 = 0;
#pragma unroll
    for (int t = 0; t < BT; ++t) {
        const uint32_t nw = l[t] & ~l0[t];
        if (nw) Lb[t * 64 + lane] = l[t];
        any |= nw;
        const uint32_t fb = pushed ? l[t] : nw;
        fany |= fb;
        fx0 |= fb & 1u;
        fx1 |= fb >> 31;
    }
    const uint32_t nt0 = pushed ? l[0] : l[0] & ~l0[0];
    const uint32_t nt1 = pushed ? l[BT - 1] : l[BT - 1] & ~l0[BT - 1];
    const bool changed = __ballot(any != 0) != 0;
    if (changed || pushed) {
        const bool fxm = __ballot(fx0 != 0) != 0, fxp = __ballot(fx1 != 0) != 0;
        const bool fym = __ballot(yl == 0 && fany) != 0, fyp = __ballot(yl == 7 && fany) != 0;
        const bool fzm = __ballot(zl == 0 && fany) != 0, fzp = __ballot(zl == 7 && fany) != 0;
        const bool ftm = __ballot(nt0 != 0) != 0, ftp = __ballot(nt1 != 0) != 0;
        if (lane == 0) {
            if (changed) {
                d.chg[par * g.NT + tile] = 1;
                d.counters[C_CHG0 + par] = 1u;
            }
            const int nx = par ^ 1;
            uint32_t nb[8];
            int k = 0;
            if (fxm && tx > 0) nb[k++] = tile - 1;
            if (fxp && tx + 1 < g.NXt) nb[k++] = tile + 1;
            if (fym && ty > 0) nb[k++] = tile - sy;
            if (fyp && ty + 1 < g.NYt) nb[k++] = tile + sy;
            if (fzm && tz > 0) nb[k++] = tile - sz;
            if (fzp && tz + 1 < g.NZt) nb[k++] = tile + sz;
            if (ftm && tt > 0) nb[k++] = tile - st;
            if (ftp && tt + 1 < g.NTt) nb[k++] = tile + st;
            schedule_batch_direct(d, nb, k, nx);
        }
    }
}

// Whether a pull tests the coupled steps in `tile`: those of tiles whose
// members changed since their last pull; with pull_all those of every tile
// that holds an admissible voxel-step (the label words of other tiles are
// left from earlier grows, never cleared).
__device__ __forceinline__ bool pull_tile(const Dev& d, const uint8_t* chg, uint32_t tile) {
    return d.pull_all ? d.active[tile] != 0 : chg[tile] != 0;
}

// Pull: a coupled particle-step joins when the voxel holding it is a member.
// Only steps in tiles whose members changed since their last pull are tested.
// A particle that gains a step is marked in pdirty for the close phase.
// Thread-level: each thread takes list entries i0, i0 + stride, ... (4 at once).
__device__ void pull_entries(const Dev& d, uint32_t i0, uint32_t stride, uint32_t n, int par) {
    const PGeom& pg = d.pg;
    const int tshift = 5 + 6 + d.g.logBT;
    const uint8_t* chg = d.chg + par * d.g.NT;
    for (uint32_t i = i0; i < n; i += 4 * stride) {
        uint2 ent[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t j = i + k * stride;
            ent[k] = j < n ? d.clist[j] : make_uint2(0u, kNoVoxel);
        }
        bool mem[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            mem[k] = ent[k].y != kNoVoxel && pull_tile(d, chg, ent[k].y >> tshift) && test_bit(d.Lf, ent[k].y);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!mem[k]) continue;
            uint32_t p, ts;
            if (pg.logTpad >= 0) {
                p = ent[k].x >> pg.logTpad;
                ts = ent[k].x & (pg.Tpad - 1);
            } else {
                p = ent[k].x / (uint32_t)pg.Tpad;
                ts = ent[k].x - p * (uint32_t)pg.Tpad;
            }
            const uint32_t wi = p * (uint32_t)pg.W + (ts >> 6);
            const unsigned long long bit = 1ull << (ts & 63);
            if (!(d.Lp[wi] & bit) && !(atomicOr(&d.Lp[wi], bit) & bit))
                atomicOr(&d.pdirty[p >> 5], 1u << (p & 31));
        }
    }
}

// Push up to N particle-steps per lane that joined (flat indices e = p * Tpad
// + t; ~0u: none): each voxel joins when admissible, for round parity `par`.
// Every step is issued for the N together (bins; activity, admissibility and
// label words; atomics; marking), and a voxel already a member takes no
// atomic.
template <int N>
__device__ void push_n(const Dev& d, const uint32_t* e, int par) {
    const Geom& g = d.g;
    uint32_t b[N];
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = e[i] != 0xFFFFFFFFu ? d.bins[e[i]] : kNoVoxel;
    uint8_t a[N];
    uint32_t aw[N], lw[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        a[i] = 0;
        aw[i] = lw[i] = 0;
        if (b[i] != kNoVoxel) {
            a[i] = d.active[b[i] >> (5 + 6 + g.logBT)];
            aw[i] = d.Af[b[i] >> 5];
            lw[i] = d.Lf[b[i] >> 5];
        }
    }
    uint32_t got[N];
    uint32_t any = kNoVoxel;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        got[i] = kNoVoxel;
        if (b[i] == kNoVoxel) continue;
        const uint32_t bit = 1u << (b[i] & 31);
        if (lw[i] & bit) continue;
        bool adm = a[i] == 1 && (aw[i] & bit);
        if (a[i] == 2) adm = in_band(d.field[voxel_of_bit(g, b[i])], d.crit[0], d.crit[1]);
        if (adm && !(atomicOr(&d.Lf[b[i] >> 5], bit) & bit)) got[i] = b[i];
        any &= got[i];
    }
    if (any != kNoVoxel) mark_voxels_n<N>(d, got, par);
}

// Push one particle-step that joined (flat index e = p * Tpad + t): its voxel
// joins when admissible, for round parity `par`.
__device__ __forceinline__ void push_one(const Dev& d, uint32_t e, int par) {
    const uint32_t b = d.bins[e];
    if (b != kNoVoxel && admissible_bit(d, b)) {
        const uint32_t bit = 1u << (b & 31);
        if (!(atomicOr(&d.Lf[b >> 5], bit) & bit)) mark_voxel(d, b, par);
    }
}

// Close one dirty particle with one label word (W = 1): its member steps
// spread over each run of admissible steps that holds them (its trajectory;
// forward in time only with forward-only coupling).  The new steps are
// returned for the caller to push.
__device__ unsigned long long close_one(const Dev& d, uint32_t p) {
    const unsigned long long a = d.Ap[p], l0 = d.Lp[p];
    const unsigned long long nw = close_word(l0, a, d.forward_only) & ~l0;
    if (nw) atomicOr(&d.Lp[p], nw);
    return nw;
}

// Lanes of one wave exchanging through LDS: order the LDS accesses around it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive prefix sum over the wave; `total` gets the wave's sum.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t& total) {
    const int lane = lane_id();
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    total = __shfl(x, 63);
    return x - v;
}

// Push the new steps of every lane of the wave (nw: new bits of label word w
// of particle p; p * Tpad + w * 64 + t is a step's flat index), 256 at a time,
// four per lane with their loads issued together.  s_list: 256 words.
__device__ void push_wave_word(const Dev& d, uint32_t p, int w, unsigned long long nw, int par,
                               uint32_t* s_list) {
    const int lane = lane_id();
    const uint32_t base = p * (uint32_t)d.pg.Tpad + (uint32_t)w * 64u;
    while (__ballot(nw != 0)) {
        uint32_t tot;
        uint32_t k = wave_excl_scan(__popcll(nw), tot);
        while (nw && k < 256) {
            s_list[k++] = base + (uint32_t)__builtin_ctzll(nw);
            nw &= nw - 1;
        }
        wave_sync();
        const uint32_t m = tot < 256 ? tot : 256;
        uint32_t e[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) e[i] = (uint32_t)lane + 64 * i < m ? s_list[lane + 64 * i] : 0xFFFFFFFFu;
        wave_sync();
        push_n<4>(d, e, par);
    }
}

// Close the dirty particles held by a wave's lanes (lane holds p when `has`)
// whose trajectories span several label words (W > 1).  Runs cross word
// boundaries, so every lane walks its words upward, carrying a run's
// membership into the next word, then downward (not with forward-only
// coupling), in step with the other lanes; after each word the wave pushes
// the steps all its lanes added, instead of each lane pushing its own steps
// one after another.
__device__ void close_words_wave(const Dev& d, uint32_t p, bool has, int par, uint32_t* s_list) {
    const int W = d.pg.W;
    unsigned long long* lw = d.Lp + (size_t)p * W;
    const unsigned long long* aw = d.Ap + (size_t)p * W;
    const int ndir = d.forward_only ? 1 : 2;
    for (int dir = 0; dir < ndir; ++dir) {
        unsigned long long carry = 0;
        for (int i = 0; i < W; ++i) {
            const int w = dir == 0 ? i : W - 1 - i;
            unsigned long long nw = 0;
            if (has) {
                const unsigned long long a = aw[w], l0 = lw[w];
                unsigned long long l;
                if (dir == 0) {
                    l = close_word(l0 | (carry & a & 1ull), a, d.forward_only);
                    carry = l >> 63;
                } else {
                    l = fill_runs64(l0 | ((carry << 63) & a), a);
                    carry = l & 1ull;
                }
                nw = l & ~l0;
                if (nw) atomicOr(&lw[w], nw);
            }
            push_wave_word(d, p, w, nw, par, s_list);
        }
    }
}

// Close phase, wave-level: the wave takes up to 64 pdirty words at a time
// (clearing them; fewer when the grid has more waves than that needs), gathers
// their dirty particles into LDS 64 at a time so that each lane closes one,
// then gathers the new steps of all its lanes so that each lane pushes one
// (several label words: word by word, four per lane).  No lane walks a long
// chain alone.  s_list: 256 words.  Returns the number of particles this wave
// closed (the same in every lane).
__device__ uint32_t close_phase(const Dev& d, int par, uint32_t wave_id, uint32_t nwaves,
                                uint32_t* s_list) {
    const PGeom& pg = d.pg;
    const uint32_t nw32 = (uint32_t)((pg.P + 31) / 32);
    const int lane = lane_id();
    // pdirty words per wave visit: up to 64, fewer when there are few words
    // per wave, so that every wave of the grid gets dirty particles
    uint32_t per = (nw32 + nwaves - 1) / nwaves;
    per = per < 1 ? 1 : (per > 64 ? 64 : per);
    uint32_t closed = 0;
    for (uint32_t base = wave_id * per; base < nw32; base += nwaves * per) {
        uint32_t wd = 0;
        if ((uint32_t)lane < per && base + lane < nw32) {
            wd = d.pdirty[base + lane];
            if (wd) d.pdirty[base + lane] = 0u;  // no setter runs during this phase
        }
        while (__ballot(wd != 0)) {
            uint32_t total;
            uint32_t k = wave_excl_scan(__popc(wd), total);
            while (wd && k < 64) {
                const int b = __ffs(wd) - 1;
                wd &= wd - 1;
                s_list[k++] = (base + lane) * 32 + b;
            }
            wave_sync();
            const uint32_t n = total < 64 ? total : 64;
            closed += n;
            uint32_t p = 0;
            const bool has = (uint32_t)lane < n;
            if (has) p = s_list[lane];
            wave_sync();
            if (pg.W > 1) {  // wave-uniform
                close_words_wave(d, p, has, par, s_list);
                continue;
            }
            unsigned long long nw = has ? close_one(d, p) : 0ull;
            while (__ballot(nw != 0)) {
                uint32_t tot2;
                uint32_t k2 = wave_excl_scan(__popcll(nw), tot2);
                while (nw && k2 < 64) {
                    const int t = __builtin_ctzll(nw);
                    nw &= nw - 1;
                    s_list[k2++] = p * (uint32_t)pg.Tpad + t;
                }
                wave_sync();
                if ((uint32_t)lane < (tot2 < 64 ? tot2 : 64)) push_one(d, s_list[lane], par);
                wave_sync();
            }
        }
    }
    return closed;
}

// OR of v over the run of consecutive lanes that hold the same key as this
// lane; the run's last lane (last = true) gets the whole run's OR.
__device__ __forceinline__ unsigned long long run_or(uint32_t key, unsigned long long v, bool& last) {
    const int lane = lane_id();
    const uint32_t kp = (uint32_t)__shfl_up((int)key, 1), kn = (uint32_t)__shfl_down((int)key, 1);
    last = lane == 63 || kn != key;
    int h = (lane == 0 || kp != key) ? lane : 0;  // lane of the run's first entry
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(h, o);
        if (lane >= o) h = max(h, y);
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(v, o);
        if (lane - o >= h) v |= y;
    }
    return v;
}

// Pull fused with close, for one 64-step label word per particle (W = 1).  A
// wave takes 64 NE list entries at a time (NE per lane); the list holds a
// particle's entries side by side, in step order.  A coupled step whose voxel
// is a member joins; the joining steps of a run of lanes holding the same
// particle are ORed into the run's last lane, which ORs their trajectory
// closure into the particle's label word with one atomic.  The label words
// only ever gain closed sets (closure distributes over union), so the bits
// that atomic sets, less the joining steps themselves (in member voxels
// already), are exactly the steps the closure adds; the lane that set them
// pushes them.  The new steps of the wave are gathered in LDS (s_list: 64 PB
// words) and pushed 64 PB at a time, PB per lane (pushes schedule for parity
// par ^ 1).  Returns this lane's number of steps joined.
template <int NE, int PB>
__device__ uint32_t pull_close_wave(const Dev& d, int par, uint32_t wave_id, uint32_t nwaves,
                                    uint32_t n, uint32_t* s_list) {
    const PGeom& pg = d.pg;
    const int tshift = 5 + 6 + d.g.logBT;
    const uint8_t* chg = d.chg + par * d.g.NT;
    const int lane = lane_id();
    uint32_t joins = 0;
    for (uint32_t base = wave_id * (64u * NE); base < n; base += nwaves * (64u * NE)) {  // wave-uniform
        uint2 ent[NE];
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const uint32_t j = base + k * 64 + lane;
            ent[k] = j < n ? d.clist[j] : make_uint2(0u, kNoVoxel);
        }
        // the label word is read only for steps in changed tiles (most are not)
        bool mem[NE];
#pragma unroll
        for (int k = 0; k < NE; ++k)
            mem[k] = ent[k].y != kNoVoxel && pull_tile(d, chg, ent[k].y >> tshift) && test_bit(d.Lf, ent[k].y);
        uint32_t pk[NE];
        unsigned long long nwk[NE];
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            pk[k] = 0;
            nwk[k] = 0ull;
            if (!__ballot(mem[k])) continue;  // wave-uniform
            const uint32_t p = pg.logTpad >= 0 ? ent[k].x >> pg.logTpad : ent[k].x / (uint32_t)pg.Tpad;
            const uint32_t ts = ent[k].x - p * (uint32_t)pg.Tpad;
            bool last;
            const unsigned long long mine =
                run_or(ent[k].y != kNoVoxel ? p : 0xFFFFFFFFu, mem[k] ? 1ull << ts : 0ull, last);
            if (!last || !mine) continue;
            if (!(mine & ~d.Lp[p])) continue;  // joined already: no atomic
            const unsigned long long cl = close_word(mine, d.Ap[p], d.forward_only);
            const unsigned long long old = atomicOr(&d.Lp[p], cl);
            joins += __popcll(mine & ~old);
            nwk[k] = cl & ~old & ~mine;
            pk[k] = p;
        }
        while (true) {
            unsigned long long anyn = 0ull;
#pragma unroll
            for (int k = 0; k < NE; ++k) anyn |= nwk[k];
            if (!__ballot(anyn != 0)) break;
            uint32_t cnt = 0;
#pragma unroll
            for (int k = 0; k < NE; ++k) cnt += __popcll(nwk[k]);
            uint32_t tot;
            uint32_t kk = wave_excl_scan(cnt, tot);
#pragma unroll
            for (int k = 0; k < NE; ++k)
                while (nwk[k] && kk < 64u * PB) {
                    const int t = __builtin_ctzll(nwk[k]);
                    nwk[k] &= nwk[k] - 1;
                    s_list[kk++] = pk[k] * (uint32_t)pg.Tpad + t;
                }
            wave_sync();
            const uint32_t m = tot < 64u * PB ? tot : 64u * PB;
            uint32_t e[PB];
#pragma unroll
            for (int i = 0; i < PB; ++i) e[i] = (uint32_t)lane + 64 * i < m ? s_list[lane + 64 * i] : 0xFFFFFFFFu;
            wave_sync();
            push_n<PB>(d, e, par ^ 1);
        }
    }
    return joins;
}

// Add a per-block value to its slot of statistic `which` (thread 0 calls).
__device__ __forceinline__ void slot_add(const Dev& d, int which, unsigned long long v) {
    if (v) atomicAdd(&d.slots[which * kSlots + (blockIdx.x & (kSlots - 1))], v);
}

// Sum a per-thread count over the block (every thread calls; uses barriers)
// and add it to the block's slot of statistic `which`.
__device__ __forceinline__ void block_slot_sum(const Dev& d, int which, uint32_t v) {
    __shared__ uint32_t s_w[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (unsigned w = 0; w < (blockDim.x + 63) / 64; ++w) t += s_w[w];
        slot_add(d, which, t);
    }
}

// ---------------------------------------------------------------------------
// Grid barrier for the persistent kernel, in two levels so that no counter
// takes an atomic from every block (same-address atomics serialise, ~12 ns
// each here): block b arrives at sub-counter b % kBarSubs; the last arrival of
// a sub-counter arrives at the top counter; the last top arrival publishes the
// barrier's epoch in a flag that every block polls.  All counters are
// monotone (epoch e expects e * n arrivals), so nothing is reset between
// barriers.  Each lives on its own 128-byte line.  The wait is bounded: after
// ~2^22 polls it records an error and returns false, so no wave can hang;
// every block then leaves the round loop.
constexpr int kBarSubs = 8;
constexpr int kBarTop = 0, kBarGen = 32, kBarSub0 = 64;  // word offsets in d.bar (kBarWords)

__device__ bool grid_sync(const Dev& d, uint32_t& epoch) {
    __shared__ uint32_t s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t e = ++epoch;
        const uint32_t j = blockIdx.x % kBarSubs;
        const uint32_t nsub = gridDim.x / kBarSubs + (j < gridDim.x % kBarSubs ? 1u : 0u);
        const uint32_t nact = gridDim.x < (uint32_t)kBarSubs ? gridDim.x : (uint32_t)kBarSubs;
        // Arrivals release; only a last arrival needs to acquire what the
        // others released before it passes them on (fence after the RMW).
        const uint32_t old = __hip_atomic_fetch_add(d.bar + kBarSub0 + 32 * j, 1u, __ATOMIC_RELEASE,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == e * nsub) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const uint32_t top = __hip_atomic_fetch_add(d.bar + kBarTop, 1u, __ATOMIC_RELEASE,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            if (top + 1 == e * nact) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(d.bar + kBarGen, e, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        uint32_t ok = 1;
        uint32_t polls = 0;
        // Poll with relaxed loads: an acquire per poll would invalidate this
        // XCD's L2 on every iteration and starve the waves still working.  One
        // acquire fence after the wait makes the other blocks' writes visible.
        while (__hip_atomic_load(d.bar + kBarGen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < e) {
            __builtin_amdgcn_s_sleep(2);
            if (++polls > (1u << 22)) {
                atomicExch(&d.counters[C_ERR], 1u);
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (load_relaxed(&d.counters[C_ERR])) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// ---------------------------------------------------------------------------
// kernels

// stat64[dst] += the slots of statistic `which`; the slots are cleared.
// Fold up to 4 slot statistics: stat64[dst[k]] (+)= the sum of slots which[k].
struct FoldList {
    int n;
    int which[4];
    int dst[4];
    int assign;
};

__device__ void fold_list(const Dev& d, const FoldList& f) {
    __shared__ unsigned long long s_w[16];
    for (int k = 0; k < f.n; ++k) {
        unsigned long long v = 0;
        for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
            v += d.slots[f.which[k] * kSlots + i];
            d.slots[f.which[k] * kSlots + i] = 0ull;
        }
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane_id() == 0) s_w[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int w = 0; w < 16; ++w) t += s_w[w];
            d.stat64[f.dst[k]] = f.assign ? t : d.stat64[f.dst[k]] + t;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_fold_slots(Dev d, FoldList f) { fold_list(d, f); }

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Zero the per-grow scheduling state in one launch.
__global__ void k_reset(Dev d) {
    const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n_dirty = 2ull * d.g.NT;
    const uint64_t n_chg = (2ull * d.g.NT + 3) / 4;
    const uint64_t n_act = ((uint64_t)d.g.NT + 3) / 4;
    const uint64_t n_pd = (uint64_t)(d.pg.P + 31) / 32;
    for (uint64_t i = tid; i < n_dirty; i += stride) d.dirty[i] = 0;
    for (uint64_t i = tid; i < n_chg; i += stride) reinterpret_cast<uint32_t*>(d.chg)[i] = 0;
    for (uint64_t i = tid; i < n_act; i += stride) reinterpret_cast<uint32_t*>(d.active)[i] = 0;
    for (uint64_t i = tid; i < n_pd; i += stride) d.pdirty[i] = 0;
    if (tid < C_NCOUNTERS) d.counters[tid] = 0;
    // the member counts (slots and statistics) belong to the read-outs, which
    // may still run for the grow before (they assign them; their folds clear
    // the slots)
    if (tid < S_NSTAT && tid != S_MEMBERS_F && tid != S_MEMBERS_P) d.stat64[tid] = 0;
    for (uint64_t i = tid; i < (uint64_t)kBarWords; i += stride) d.bar[i] = 0;
    for (uint64_t i = tid; i < (uint64_t)kSlotStats * kSlots; i += stride) {
        const uint64_t row = i / kSlots;
        if (row != SL_MEMBERS_F && row != SL_MEMBERS_P) d.slots[i] = 0ull;
    }
    for (uint64_t i = tid; i < 2ull * kWorkSubs; i += stride) d.wcnt[i * kWcntStride] = 0u;
}

// Load: bin every particle-step into the voxel covering it (at the field step
// holding the step's time, t / tr) and transpose the values to particle-major
// rows.  Block = 64 particles; LDS tile [64][65].
__global__ __launch_bounds__(256) void k_bin_particles(Geom g, PGeom pg,
                                                       const float* __restrict__ xyz,
                                                       const float* __restrict__ attr,
                                                       uint32_t* __restrict__ bins,
                                                       float* __restrict__ attr_t) {
    __shared__ uint32_t sb[64][65];
    __shared__ float sa[64][65];
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const int TC = pg.Tpad < 64 ? pg.Tpad : 64;
    for (int t0 = 0; t0 < pg.Tpad; t0 += TC) {
        for (int i = threadIdx.x; i < 64 * TC; i += blockDim.x) {
            const int pl = i & 63, tl = i >> 6;
            const int64_t p = p0 + pl;
            const int t = t0 + tl;
            uint32_t b = kNoVoxel;
            float a = __builtin_nanf("");
            if (p < pg.P && t < pg.T) {
                const float* q = xyz + ((int64_t)t * pg.P + p) * 3;
                const float cx = floorf(q[0]), cy = floorf(q[1]), cz = floorf(q[2]);
                if (cx >= 0.0f && cx < (float)g.X && cy >= 0.0f && cy < (float)g.Y &&
                    cz >= 0.0f && cz < (float)g.Z)
                    b = bit_index(g, (int)cx, (int)cy, (int)cz, t / pg.tr);
                a = attr[(int64_t)t * pg.P + p];
            }
            sb[pl][tl] = b;
            sa[pl][tl] = a;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * TC; i += blockDim.x) {
            const int pl = i / TC, tl = i - pl * TC;
            const int64_t p = p0 + pl;
            if (p < pg.P) {
                const int64_t e = p * pg.Tpad + t0 + tl;
                bins[e] = sb[pl][tl];
                attr_t[e] = sa[pl][tl];
            }
        }
        __syncthreads();
    }
}

typedef float v4f __attribute__((ext_vector_type(4)));

// Admissibility of every voxel-step, bit-packed into tiles, and the labels
// cleared.  Block = 256 threads for the 64 rows (z_l, y_l) of one (t, tz, ty);
// x in passes of 256.  Each lane tests 4 consecutive x (one 16-byte
// non-temporal load); 8 lanes OR their nibbles into one word.
__global__ __launch_bounds__(256) void k_admit_field(Dev d) {
    __shared__ uint32_t sw[8 * 64];
    const Geom& g = d.g;
    const float lo = d.crit[0], hi = d.crit[1];
    const int ty = blockIdx.x, tz = blockIdx.y, t = blockIdx.z;
    const int tt = t >> g.logBT, tl = t & (g.BT - 1);
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const bool vec = (g.X & 3) == 0;
    for (int tx0 = 0; tx0 < g.NXt; tx0 += 8) {
        const int ntx = min(8, g.NXt - tx0);
        const int x = tx0 * 32 + 4 * lane;
        v4f v[16];
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int row = wave * 16 + rr;
            const int y = ty * 8 + (row & 7), z = tz * 8 + (row >> 3);
            const float nan = __builtin_nanf("");
            v[rr] = (v4f){nan, nan, nan, nan};
            if (y < g.Y && z < g.Z) {
                const float* rp = d.field + ((size_t)(t * g.Z + z) * g.Y + y) * g.X;
                if (vec) {
                    if (x < g.X)
                        v[rr] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(rp + x));
                } else {
                    if (x < g.X) v[rr].x = rp[x];
                    if (x + 1 < g.X) v[rr].y = rp[x + 1];
                    if (x + 2 < g.X) v[rr].z = rp[x + 2];
                    if (x + 3 < g.X) v[rr].w = rp[x + 3];
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int row = wave * 16 + rr;
            const uint32_t nib = (uint32_t)in_band(v[rr].x, lo, hi) |
                                 ((uint32_t)in_band(v[rr].y, lo, hi) << 1) |
                                 ((uint32_t)in_band(v[rr].z, lo, hi) << 2) |
                                 ((uint32_t)in_band(v[rr].w, lo, hi) << 3);
            uint32_t w = nib << (4 * (lane & 7));
            w |= __shfl_xor(w, 1);
            w |= __shfl_xor(w, 2);
            w |= __shfl_xor(w, 4);
            if ((lane & 7) == 0 && (lane >> 3) < ntx) sw[(lane >> 3) * 64 + row] = w;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < ntx * 64; i += 256) {
            const int txl = i >> 6, row = i & 63;
            const uint32_t tile = tile_of(g, tx0 + txl, ty, tz, tt);
            const uint32_t w = sw[i];
            const size_t wi = (size_t)tile * g.WPT + tl * 64 + row;
            d.Af[wi] = w;
            d.Lf[wi] = 0u;
            if (__ballot(w != 0) != 0 && lane == 0) d.active[tile] = 1;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void minmax_skip_nan(float v, float& mn, float& mx) {
    if (v == v) {
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
}

// Load time: (min, max) of each tile's non-NaN field values ((+inf, -inf)
// when it has none).  A tile can hold a voxel with lo <= f <= hi only if
// max >= lo and min <= hi, so these decide, exactly, which tiles a grow must
// test at all.  Block = one tile, wave = t-slices; when X is a multiple of 4
// eight lanes read one 128-byte tile row with 16-byte loads, so a wave
// instruction covers 8 whole rows.
__global__ __launch_bounds__(256) void k_tile_summaries(Geom g, const float* __restrict__ f,
                                                        float2* __restrict__ tsum) {
    __shared__ float s_mn[4], s_mx[4];
    const uint32_t tile = blockIdx.x;
    int tx, ty, tz, tt;
    tile_coords(g, tile, tx, ty, tz, tt);
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    float mn = __builtin_inff(), mx = -__builtin_inff();
    if ((g.X & 3) == 0) {
        const int quad = lane & 7;
        const int x = tx * 32 + quad * 4;
        for (int tl = wave; tl < g.BT; tl += 4) {
            const int t = (tt << g.logBT) + tl;
            if (t >= g.T) break;
            v4f v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int row = i * 8 + (lane >> 3);  // (z_l, y_l) = (row >> 3, row & 7)
                const int y = ty * 8 + (row & 7), z = tz * 8 + (row >> 3);
                v[i] = (v4f){__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf("")};
                if (x < g.X && y < g.Y && z < g.Z)
                    v[i] = __builtin_nontemporal_load(
                        reinterpret_cast<const v4f*>(f + ((size_t)(t * g.Z + z) * g.Y + y) * g.X + x));
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                minmax_skip_nan(v[i].x, mn, mx);
                minmax_skip_nan(v[i].y, mn, mx);
                minmax_skip_nan(v[i].z, mn, mx);
                minmax_skip_nan(v[i].w, mn, mx);
            }
        }
    } else {
        const int xl = lane & 31;
        const int x = tx * 32 + xl;
        for (int tl = wave; tl < g.BT; tl += 4) {
            const int t = (tt << g.logBT) + tl;
            if (t >= g.T) break;
            for (int row = lane >> 5; row < 64; row += 2) {
                const int y = ty * 8 + (row & 7), z = tz * 8 + (row >> 3);
                if (x < g.X && y < g.Y && z < g.Z)
                    minmax_skip_nan(f[((size_t)(t * g.Z + z) * g.Y + y) * g.X + x], mn, mx);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, o));
        mx = fmaxf(mx, __shfl_xor(mx, o));
    }
    if (lane == 0) {
        s_mn[wave] = mn;
        s_mx[wave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        tsum[tile] = make_float2(fminf(fminf(s_mn[0], s_mn[1]), fminf(s_mn[2], s_mn[3])),
                                 fmaxf(fmaxf(s_mx[0], s_mx[1]), fmaxf(s_mx[2], s_mx[3])));
}

// Load time: (min, max) of each particle's non-NaN values over its steps
// (padding steps hold NaN).  A group of G lanes reads one particle's row with
// 16-byte loads (G = 16, or Tpad / 4 for short rows), so a wave instruction
// covers whole rows.
__global__ __launch_bounds__(256) void k_particle_summaries(PGeom pg, const float* __restrict__ at,
                                                            float2* __restrict__ psum) {
    if (pg.Tpad < 4) {
        for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < pg.P;
             p += (int64_t)gridDim.x * blockDim.x) {
            float mn = __builtin_inff(), mx = -__builtin_inff();
            for (int t = 0; t < pg.Tpad; ++t) minmax_skip_nan(at[p * pg.Tpad + t], mn, mx);
            psum[p] = make_float2(mn, mx);
        }
        return;
    }
    const int G = pg.Tpad >= 64 ? 16 : (pg.Tpad >> 2);
    const int per_wave = 64 / G;
    const int lane = lane_id(), sub = lane & (G - 1);
    const int64_t wave_id = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int nq = pg.Tpad >> 2;
    for (int64_t p0 = wave_id * per_wave; p0 < pg.P; p0 += nwaves * per_wave) {
        const int64_t p = p0 + lane / G;
        float mn = __builtin_inff(), mx = -__builtin_inff();
        if (p < pg.P) {
            const v4f* row = reinterpret_cast<const v4f*>(at + p * pg.Tpad);
            for (int c = sub; c < nq; c += G) {
                const v4f v = __builtin_nontemporal_load(row + c);
                minmax_skip_nan(v.x, mn, mx);
                minmax_skip_nan(v.y, mn, mx);
                minmax_skip_nan(v.z, mn, mx);
                minmax_skip_nan(v.w, mn, mx);
            }
        }
        for (int o = 1; o < G; o <<= 1) {
            mn = fminf(mn, __shfl_xor(mn, o));
            mx = fmaxf(mx, __shfl_xor(mx, o));
        }
        if (p < pg.P && sub == 0) psum[p] = make_float2(mn, mx);
    }
}

// Tiles whose value range meets the field band, as a list.
__global__ __launch_bounds__(256) void k_tile_candidates(Dev d) {
    __shared__ uint32_t s_tmp[8];
    const float lo = d.crit[0], hi = d.crit[1];
    for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < d.g.NT; b0 += gridDim.x * blockDim.x) {
        const uint32_t i = b0 + threadIdx.x;
        bool c = false;
        if (i < d.g.NT) {
            const float2 r = d.tsum[i];
            c = r.y >= lo && r.x <= hi;
        }
        const uint32_t k = block_append256(c ? 1u : 0u, &d.counters[C_NCAND], s_tmp);
        if (c) d.cand[k] = i;
    }
}

// Admissibility of the voxel-steps of candidate tiles, and their labels
// cleared.  Block = one tile at a time; each wave handles t-slices, each lane
// one (z_l, y_l) row of 32 x.  With a predictor, candidates it does not mark
// are only cleared and deferred to the first sweep that reaches them.
__global__ __launch_bounds__(256) void k_admit_tiles(Dev d) {
    const Geom& g = d.g;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t n = d.counters[C_NCAND];
    uint32_t tested = 0, active = 0;  // this block's counts (thread 0)
    for (uint32_t ci = blockIdx.x; ci < n; ci += gridDim.x) {
        const uint32_t tile = d.cand[ci];
        int tx, ty, tz, tt;
        tile_coords(g, tile, tx, ty, tz, tt);
        const bool defer = d.tpred && !d.tpred[tile];
        uint32_t any = 0;
        for (int tl = wave; tl < g.BT; tl += 4) {
            const size_t wi = (size_t)tile * g.WPT + tl * 64 + lane;
            if (!defer) {
                const uint32_t w = slice_admissibility(d, tx, ty, tz, (tt << g.logBT) + tl);
                d.Af[wi] = w;
                any |= w;
            }
            d.Lf[wi] = 0u;
        }
        if (defer) {
            if (threadIdx.x == 0) {
                d.active[tile] = 2;
                ++active;
            }
            continue;
        }
        const bool has = __ballot(any != 0) != 0;
        if (has && lane == 0) d.active[tile] = 1;  // each wave's lane 0: the same value
        // the block's waves may disagree: count the tile once, from all waves
        __shared__ uint32_t s_any;
        if (threadIdx.x == 0) s_any = 0;
        __syncthreads();
        if (has && lane == 0) s_any = 1;
        __syncthreads();
        if (threadIdx.x == 0) {
            ++tested;
            active += s_any;
        }
    }
    if (threadIdx.x == 0) {
        slot_add(d, SL_TESTED, tested);
        slot_add(d, SL_ACTIVE, active);
    }
}

__global__ __launch_bounds__(256) void k_count_active(Dev d) {
    uint32_t c = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < d.g.NT;
         i += gridDim.x * blockDim.x)
        c += d.active[i] != 0;
    block_slot_sum(d, SL_ACTIVE, c);
}

// Admissibility of every particle-step, the labels cleared, and the coupled
// list: every admissible particle-step that lies in a voxel, as (flat index,
// voxel bit).  Lanes load 4 consecutive steps (16 bytes, non-temporal); the
// lanes covering one label word (up to 64 steps) OR their nibbles together; a
// lane with an admissible step loads the 4 matching bins (16 bytes).  Entries
// are staged in LDS and flushed to the global list with one atomic per flush
// (one per block at config 3): appends to a single counter from every block
// serialise, so their number, not the bytes, sets this kernel's time.
// Requires Tpad >= 4.
constexpr uint32_t kStage = 1024;  // staged entries per block (8 KB of LDS)
__device__ __forceinline__ void flush_stage(const Dev& d, const uint2* s_buf, uint32_t n, uint32_t* s_tmp) {
    if (threadIdx.x == 0) s_tmp[8] = atomicAdd(&d.counters[C_NLIST], n);
    __syncthreads();
    const uint32_t base = s_tmp[8];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) d.clist[base + i] = s_buf[i];
    __syncthreads();
}

// Admissibility of the candidate particles' steps, their labels cleared, and
// the coupled list: every admissible particle-step that lies in a voxel, as
// (flat index, voxel bit).  A unit is one 64-step label word of a candidate
// (or a whole row when Tpad < 64); G lanes read it with 16-byte loads and OR
// their nibbles into the word.  A lane with an admissible step loads the 4
// matching bins (16 bytes).  Entries are staged in LDS and flushed to the
// global list with one atomic per flush (appends to one counter from every
// block serialise).  Non-candidates are not touched: their pflag is 0.
// Requires Tpad >= 4.
//
// The candidates are found in the same pass: a block takes kAdmitChunk
// particles at a time (four consecutive ones per thread), flags those whose
// load-time value range meets the band (pflag), lists them in index order in
// LDS and then tests their units; the coupled list keeps each particle's
// entries side by side in step order.
constexpr int kAdmitChunk = 1024;
__global__ __launch_bounds__(256) void k_admit_particles(Dev d) {
    __shared__ __align__(8) uint32_t s_tmp[10];
    __shared__ uint2 s_buf[kStage];
    __shared__ uint32_t s_cand[kAdmitChunk];
    const PGeom& pg = d.pg;
    const float lo = d.crit[2], hi = d.crit[3];
    const int G = pg.Tpad >= 64 ? 16 : (pg.Tpad >> 2);  // lanes per unit (power of two)
    const uint32_t upb = 256 / G;                       // units per block pass
    const int W = pg.W;
    const int sub = threadIdx.x & (G - 1);
    const v4f* src = reinterpret_cast<const v4f*>(d.attr_t);
    const uint4* bsrc = reinterpret_cast<const uint4*>(d.bins);
    uint32_t nbuf = 0;  // entries staged; the same in every thread
    for (int64_t c0 = (int64_t)blockIdx.x * kAdmitChunk; c0 < pg.P;
         c0 += (int64_t)gridDim.x * kAdmitChunk) {  // block-uniform
        uint32_t flags = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t p = c0 + 4 * threadIdx.x + j;
            if (p < pg.P) {
                const float2 r = d.psum[p];
                const bool in = r.y >= lo && r.x <= hi;
                d.pflag[p] = in ? 1 : 0;
                flags |= (in ? 1u : 0u) << j;
            }
        }
        uint32_t ncand;  // the same in every thread
        uint32_t at = block_exclusive_scan256((uint32_t)__popc(flags), s_tmp, ncand);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((flags >> j) & 1u) s_cand[at++] = (uint32_t)(c0 + 4 * threadIdx.x + j);
        __syncthreads();
        const uint32_t nunits = ncand * (uint32_t)W;
        for (uint32_t ub = 0; ub < nunits; ub += 4 * upb) {  // block-uniform
            v4f v[4];
            uint32_t e0[4], wi[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t u = ub + k * upb + threadIdx.x / G;
                const float nan = __builtin_nanf("");
                v[k] = (v4f){nan, nan, nan, nan};
                e0[k] = 0xFFFFFFFFu;
                if (u < nunits) {
                    const uint32_t p = s_cand[W == 1 ? u : u / W];
                    const uint32_t w = W == 1 ? 0u : (uint32_t)(u % W);
                    e0[k] = p * (uint32_t)pg.Tpad + w * 64u + (uint32_t)sub * 4u;
                    wi[k] = p * (uint32_t)W + w;
                    v[k] = __builtin_nontemporal_load(src + (e0[k] >> 2));
                }
            }
            uint32_t nibs[4];
            uint4 bn[4];
            uint32_t cnt = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t nib = (uint32_t)in_band(v[k].x, lo, hi) |
                                     ((uint32_t)in_band(v[k].y, lo, hi) << 1) |
                                     ((uint32_t)in_band(v[k].z, lo, hi) << 2) |
                                     ((uint32_t)in_band(v[k].w, lo, hi) << 3);
                unsigned long long x = (unsigned long long)nib << (4 * sub);
                for (int o = 1; o < G; o <<= 1) x |= __shfl_xor(x, o);
                if (sub == 0 && e0[k] != 0xFFFFFFFFu) {
                    d.Ap[wi[k]] = x;
                    d.Lp[wi[k]] = 0ull;
                }
                bn[k] = make_uint4(kNoVoxel, kNoVoxel, kNoVoxel, kNoVoxel);
                if (nib) bn[k] = bsrc[e0[k] >> 2];  // nib != 0 implies a unit in range
                uint32_t m = nib;
                if (bn[k].x == kNoVoxel) m &= ~1u;
                if (bn[k].y == kNoVoxel) m &= ~2u;
                if (bn[k].z == kNoVoxel) m &= ~4u;
                if (bn[k].w == kNoVoxel) m &= ~8u;
                nibs[k] = m;
                cnt += __popc(m);
            }
            // Positions: the entries of unit set k of every thread come before
            // those of set k + 1, in thread order within a set, so that the
            // entries of one unit (its G lanes) are contiguous and in step order
            // (the pull combines a particle's entries that sit side by side).
            // Four 16-bit counts scanned in one 64-bit word.
            unsigned long long packed = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) packed |= (unsigned long long)__popc(nibs[k]) << (16 * k);
            unsigned long long tot64;
            const unsigned long long ex64 = block_exclusive_scan256_u64(packed, s_tmp, tot64);
            uint32_t setbase[4], total = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                setbase[k] = total;
                total += (uint32_t)(tot64 >> (16 * k)) & 0xFFFFu;
            }
            (void)cnt;
            if (nbuf + total > kStage) {  // block-uniform
                flush_stage(d, s_buf, nbuf, s_tmp);
                nbuf = 0;
            }
            const bool direct = total > kStage;  // block-uniform; more than the stage holds
            uint32_t base = nbuf;
            if (direct) {
                if (threadIdx.x == 0) s_tmp[8] = atomicAdd(&d.counters[C_NLIST], total);
                __syncthreads();
                base = s_tmp[8];
                __syncthreads();
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!nibs[k]) continue;
                uint32_t out = base + setbase[k] + ((uint32_t)(ex64 >> (16 * k)) & 0xFFFFu);
                const uint32_t bw[4] = {bn[k].x, bn[k].y, bn[k].z, bn[k].w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (!((nibs[k] >> j) & 1u)) continue;
                    const uint2 e = make_uint2(e0[k] + j, bw[j]);
                    if (direct) d.clist[out++] = e;
                    else s_buf[out++] = e;
                }
            }
            if (!direct) nbuf += total;
        }
        __syncthreads();  // every unit of the chunk read its candidate before the next list
    }
    if (nbuf) flush_stage(d, s_buf, nbuf, s_tmp);
}

// Same for Tpad < 4 (T <= 2): one thread per particle.
__global__ void k_admit_particles_short(Dev d) {
    const PGeom& pg = d.pg;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < pg.P;
         p += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long x = 0;
        for (int t = 0; t < pg.Tpad; ++t)
            if (in_band(d.attr_t[p * pg.Tpad + t], d.crit[2], d.crit[3])) x |= 1ull << t;
        d.Ap[p] = x;
        d.Lp[p] = 0ull;
        d.pflag[p] = 1;
    }
}

// Coupled list for short rows (Tpad < 4): every admissible particle-step that
// lies in a voxel, as (flat index, voxel bit); one thread per label word, one
// atomic per block.
__global__ __launch_bounds__(256) void k_couple(Dev d) {
    __shared__ uint32_t s_tmp[8];
    const PGeom& pg = d.pg;
    const uint64_t nw = (uint64_t)pg.P * pg.W;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b0 = blockIdx.x * (uint64_t)blockDim.x; b0 < nw; b0 += stride) {
        const uint64_t i = b0 + threadIdx.x;
        const unsigned long long m = i < nw ? d.Ap[i] : 0ull;
        const uint64_t p = pg.W == 1 ? i : i / pg.W;
        const uint32_t t0 = pg.W == 1 ? 0u : (uint32_t)(i - p * pg.W) * 64u;
        const uint32_t* row = d.bins + p * pg.Tpad + t0;
        uint32_t cnt = 0;
        for (unsigned long long r = m; r; r &= r - 1) cnt += row[__builtin_ctzll(r)] != kNoVoxel;
        uint32_t k = block_append256(cnt, &d.counters[C_NLIST], s_tmp);
        for (unsigned long long r = m; r; r &= r - 1) {
            const int t = __builtin_ctzll(r);
            const uint32_t b = row[t];
            if (b != kNoVoxel) d.clist[k++] = make_uint2((uint32_t)(p * pg.Tpad + t0 + t), b);
        }
    }
}

__global__ void k_seeds(Dev d, const int32_t* __restrict__ seeds, int64_t S) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= S) return;
    const int32_t* s = seeds + 4 * i;
    const uint32_t b = bit_index(d.g, s[0], s[1], s[2], s[3]);
    if (admissible_bit(d, b)) {
        const uint32_t bit = 1u << (b & 31);
        if (!(atomicOr(&d.Lf[b >> 5], bit) & bit)) mark_voxel(d, b, 0);
    } else {
        atomicAdd(&d.counters[C_DROPPED], 1u);
    }
}

// ---------------------------------------------------------------------------
// score-ordered schedulers (learned and heuristic priority)

__device__ __forceinline__ uint32_t score_key(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Sort keys of the candidate tiles (value range meets the band): the
// order-preserving bits of the tile's score when the score reaches thr, else
// 0; value = the tile.  Score: with logits ([T][Db][Hb][Wb] over 8^3-voxel
// brick-steps) the largest logit of the tile's brick-steps, else the tile's
// greatest field value.  count: tiles with a nonzero key.
__global__ void k_priority_keys(Dev d, const float* __restrict__ logits, int bW, int bH, int bD, float thr,
                                uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t* count) {
    const Geom& g = d.g;
    const float lo = d.crit[0], hi = d.crit[1];
    for (uint32_t tile = blockIdx.x * blockDim.x + threadIdx.x; tile < g.NT; tile += gridDim.x * blockDim.x) {
        const float2 r = d.tsum[tile];
        uint32_t key = 0;
        if (r.y >= lo && r.x <= hi) {
            float score = r.y;
            if (logits) {
                int tx, ty, tz, tt;
                tile_coords(g, tile, tx, ty, tz, tt);
                score = -INFINITY;
                for (int tl = 0; tl < g.BT; ++tl) {
                    const int t = (tt << g.logBT) + tl;
                    if (t >= g.T) break;
                    for (int k = 0; k < 4; ++k) {
                        const int bx = tx * 4 + k;
                        if (bx >= bW) break;
                        const float v = logits[(((size_t)t * bD + tz) * bH + ty) * bW + bx];
                        score = v > score ? v : score;  // NaN logits never raise it
                    }
                }
            }
            if (score >= thr) key = score_key(score);
        }
        keys[tile] = key;
        vals[tile] = tile;
        if (key) atomicAdd(count, 1u);
    }
}

// The priority pass: the first count tiles of `list` (descending score) are
// swept in list order by nwaves waves, wave w taking items w, w + nwaves, ...
// so that a tile later in the list sees what earlier ones set (Gauss-Seidel
// within the pass).  Sweeps schedule the tiles across faces that gained bits
// into the work list of parity par ^ 1, as in a round of parity par.
template <int BT>
__global__ __launch_bounds__(256) void k_priority_sweep(Dev d, const uint32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ count, int par) {
    const uint32_t wave0 = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t n = *count;
    for (uint32_t w = wave0; w < n; w += nwaves) {
        const uint32_t tile = list[w];
        if (d.active[tile] == 1) sweep_tile<BT>(d, tile, par);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&d.stat64[S_PRIO_VISITS], (unsigned long long)n);
}

// The verification round's schedule: every tile holding an admissible
// voxel-step on the work list of parity par.  Its "changed" flag is left
// alone: the round sweeps each tile as an ordinary visit (only faces that
// gain bits schedule a neighbour), and its pull tests every coupled step
// (Dev::pull_all) instead of those of changed tiles.
__global__ __launch_bounds__(256) void k_verify_schedule(Dev d, int par) {
    for (uint32_t t0 = blockIdx.x * blockDim.x; t0 < d.g.NT; t0 += gridDim.x * blockDim.x) {
        const uint32_t tile = t0 + threadIdx.x;
        uint32_t nb[1] = {tile};
        const int k = tile < d.g.NT && d.active[tile] == 1 ? 1 : 0;
        schedule_batch(d, nb, k, par);
    }
}

// ---------------------------------------------------------------------------
// Jacobi sweeps (a debugging schedule): X_{k+1} = X_k with every admissible
// node one edge away from X_k added, computed from X_k alone (read from the
// current label arrays, written to the next ones).  From the admissible
// seeds, the sweep that adds nothing is number D + 1, D the largest
// breadth-first level of the grown set.

// Label word of the row (y, z, t) of x-tile tx, or 0 outside the tile grid.
__device__ __forceinline__ uint32_t jword(const Geom& g, const uint32_t* L, int tx, int y, int z, int t) {
    if (tx < 0 || tx >= g.NXt || y < 0 || y >= g.NYt * 8 || z < 0 || z >= g.NZt * 8 || t < 0 ||
        t >= (g.NTt << g.logBT))
        return 0u;
    const uint32_t tile = tile_of(g, tx, y >> 3, z >> 3, t >> g.logBT);
    return L[(size_t)tile * g.WPT + (((t & (g.BT - 1)) * 8 + (z & 7)) * 8 + (y & 7))];
}

// Field edges: each word of the next labels = its current word plus the
// admissible bits with a member neighbour (x within and across words, y, z,
// t from the neighbouring rows).
__global__ __launch_bounds__(256) void k_jacobi_field(Dev d, const uint32_t* __restrict__ cur,
                                                      uint32_t* __restrict__ nxt) {
    const Geom& g = d.g;
    for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < g.nwords;
         w += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = cur[w];
        const uint32_t a = d.Af[w];
        uint32_t add = 0;
        if (a & ~c) {
            const uint32_t tile = (uint32_t)(w / g.WPT), wi = (uint32_t)(w % g.WPT);
            int tx, ty, tz, tt;
            tile_coords(g, tile, tx, ty, tz, tt);
            const int y = ty * 8 + (wi & 7), z = tz * 8 + ((wi >> 3) & 7), t = (tt << g.logBT) + (wi >> 6);
            uint32_t n = (c << 1) | (c >> 1);
            n |= jword(g, cur, tx - 1, y, z, t) >> 31;
            n |= jword(g, cur, tx + 1, y, z, t) << 31;
            n |= jword(g, cur, tx, y - 1, z, t) | jword(g, cur, tx, y + 1, z, t);
            n |= jword(g, cur, tx, y, z - 1, t) | jword(g, cur, tx, y, z + 1, t);
            n |= jword(g, cur, tx, y, z, t - 1) | jword(g, cur, tx, y, z, t + 1);
            add = n & a & ~c;
        }
        if (add) {
            atomicOr(&nxt[w], add);
            d.counters[C_JCHANGED] = 1u;
        }
    }
}

// Particle edges, one thread per particle-step of the candidate particles:
// a member step puts its admissible voxel into the next labels; a
// non-member admissible step joins when its voxel or the same particle at t -
// 1 (or t + 1, unless coupling is forward-only) is a member now.
__global__ __launch_bounds__(256) void k_jacobi_particles(Dev d, const uint32_t* __restrict__ lf_cur,
                                                          const unsigned long long* __restrict__ lp_cur,
                                                          uint32_t* __restrict__ lf_nxt,
                                                          unsigned long long* __restrict__ lp_nxt) {
    const PGeom& pg = d.pg;
    const uint64_t n = (uint64_t)pg.P * pg.Tpad;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = e / pg.Tpad;
        const int t = (int)(e - p * pg.Tpad);
        if (t >= pg.T || !d.pflag[p]) continue;
        auto member = [&](int s) -> bool {
            return (lp_cur[p * pg.W + (s >> 6)] >> (s & 63)) & 1ull;
        };
        const uint32_t b = d.bins[e];
        if (member(t)) {
            if (b != kNoVoxel && test_bit(d.Af, b) && !test_bit(lf_cur, b)) {
                atomicOr(&lf_nxt[b >> 5], 1u << (b & 31));
                d.counters[C_JCHANGED] = 1u;
            }
            continue;
        }
        if (!((d.Ap[p * pg.W + (t >> 6)] >> (t & 63)) & 1ull)) continue;
        const bool join = (b != kNoVoxel && test_bit(lf_cur, b)) || (t > 0 && member(t - 1)) ||
                          (!d.forward_only && t + 1 < pg.T && member(t + 1));
        if (join) {
            atomicOr(&lp_nxt[p * pg.W + (t >> 6)], 1ull << (t & 63));
            d.counters[C_JCHANGED] = 1u;
        }
    }
}

// Sweep every tile on the work list of parity `par` (its kWorkSubs sub-lists
// read as one list: lane j holds sub-list j's length and prefix, so a wave
// finds the sub-list of flat index w with one ballot).  Returns the list's
// length (the same in every lane).
template <int BT>
__device__ uint32_t sweep_phase(const Dev& d, int par, uint32_t wave0, uint32_t nwaves) {
    const int lane = lane_id();
    const uint32_t cj = load_relaxed(&d.wcnt[(par * kWorkSubs + lane) * kWcntStride]);
    uint32_t total;
    const uint32_t ex = wave_excl_scan(cj, total);
    for (uint32_t w = wave0; w < total; w += nwaves) {
        const uint32_t j = (uint32_t)__popcll(__ballot(ex + cj <= w));  // sub-lists wholly before w
        const uint32_t k = w - (uint32_t)__shfl((int)ex, (int)j);
        sweep_tile<BT>(d, d.work[(size_t)(par * kWorkSubs + j) * d.g.WCAP + k], par);
    }
    return total;
}

// Sum the sub-list lengths of parity `par` into the host-visible counter.
__global__ void k_work_total(Dev d, int par) {
    uint32_t total;
    wave_excl_scan(d.wcnt[(par * kWorkSubs + lane_id()) * kWcntStride], total);
    if (threadIdx.x == 0) d.counters[C_NWORK0 + par] = total;
}

// End of a chunk of rounds: the work total (first wave), a copy of the round
// count and that total for the read-outs' gate (snap: C_NCOUNTERS words, not
// touched by later grows' rounds), and the statistics fold.
__global__ __launch_bounds__(1024) void k_chunk_end(Dev d, int par, FoldList f, uint32_t* snap) {
    if (threadIdx.x < 64) {
        uint32_t total;
        wave_excl_scan(d.wcnt[(par * kWorkSubs + lane_id()) * kWcntStride], total);
        if (threadIdx.x == 0) {
            d.counters[C_NWORK0 + par] = total;
            if (snap) {
                snap[C_NWORK0 + par] = total;
                snap[C_ROUNDS] = d.counters[C_ROUNDS];
            }
        }
    }
    fold_list(d, f);
}

// ---- one round as three launches ----

template <int BT>
__global__ __launch_bounds__(256) void k_round_sweep(Dev d, int par) {
    const uint32_t wave0 = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    // the other parity's changed-tile flags were consumed by the previous
    // round's pull; clear them before this round's pull pushes set them again
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < d.g.NT; i += gridDim.x * blockDim.x)
        d.chg[(par ^ 1) * d.g.NT + i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) d.counters[C_CHG0 + (par ^ 1)] = 0u;
    const uint32_t nwork = sweep_phase<BT>(d, par, wave0, nwaves);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.counters[C_RACT] = nwork ? 1u : 0u;  // pull and close of this round read it
        if (nwork) {
            d.counters[C_ROUNDS] += 1u;
            // every listed tile is swept once: the visit count is the list length
            atomicAdd(&d.stat64[S_TILE_VISITS], (unsigned long long)nwork);
        }
    }
}

__global__ __launch_bounds__(256) void k_round_pull(Dev d, int par) {
    __shared__ uint32_t s_list[4 * 256];
    if (!d.counters[C_RACT]) return;
    // the swept list is empty again (its dirty flags were cleared by the sweeps)
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)kWorkSubs)
        d.wcnt[(par * kWorkSubs + threadIdx.x) * kWcntStride] = 0u;
    // no tile's members changed since the last pull (set flags raise the
    // parity's flag word): nothing can join
    if (!d.pull_all && !d.counters[C_CHG0 + par]) return;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = d.counters[C_NLIST];
    if (d.pg.W == 1) {
        const uint32_t joins =
            pull_close_wave<4, 4>(d, par, tid >> 6, (gridDim.x * blockDim.x) >> 6, n, s_list + 256 * (threadIdx.x >> 6));
        block_slot_sum(d, SL_PART_VISITS, joins);
    } else {
        pull_entries(d, tid, gridDim.x * blockDim.x, n, par);
    }
}

__global__ __launch_bounds__(256) void k_round_close(Dev d, int par) {
    __shared__ uint32_t s_list[4 * 256];
    __shared__ uint32_t s_cnt;
    if (!d.counters[C_RACT]) return;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const uint32_t closed =
        close_phase(d, par ^ 1, tid >> 6, stride >> 6, s_list + 256 * (threadIdx.x >> 6));
    if (lane_id() == 0 && closed) atomicAdd(&s_cnt, closed);
    __syncthreads();
    if (threadIdx.x == 0) slot_add(d, SL_PART_VISITS, s_cnt);
}

// ---- all rounds in one cooperative launch ----
// Pull entries and pushes per lane per wave step inside the persistent kernel:
// its grid (two blocks per CU) has a quarter of the waves a launched pull has,
// so each wave takes more entries at once, and pushes more at once, instead of
// running the chain of round trips several times over.
constexpr int kCoopNE = 8;

template <int BT>
__global__ __launch_bounds__(256) void k_rounds(Dev d, uint32_t round0, uint32_t max_rounds) {
    __shared__ uint32_t s_list[4 * 64 * kCoopNE];
    __shared__ uint32_t s_cnt;
    uint32_t epoch = 0;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nthreads = gridDim.x * blockDim.x;
    const uint32_t wave0 = tid >> 6, nwaves = nthreads >> 6;
    const bool parts = d.pg.P > 0;
    uint32_t* my_list = s_list + 64 * kCoopNE * (threadIdx.x >> 6);
    if (threadIdx.x == 0) s_cnt = 0;
    uint32_t r = round0;
    uint32_t visits = 0, closed = 0;
    uint32_t nwork = 0;
    while (true) {
        const int par = r & 1;
        {
            uint32_t total;
            wave_excl_scan(load_relaxed(&d.wcnt[(par * kWorkSubs + lane_id()) * kWcntStride]), total);
            nwork = total;  // the same in every thread
        }
        if (nwork == 0 || (max_rounds && r - round0 >= max_rounds)) break;
        // sweep (and clear the flags the previous round's pull consumed)
        for (uint32_t i = tid; i < d.g.NT; i += nthreads) d.chg[(par ^ 1) * d.g.NT + i] = 0;
        sweep_phase<BT>(d, par, wave0, nwaves);
        visits += nwork;  // only thread 0 records it
        if (!grid_sync(d, epoch)) break;
        // pull (fused with close and push for one label word per particle)
        if (tid < (unsigned)kWorkSubs) store_relaxed(&d.wcnt[(par * kWorkSubs + tid) * kWcntStride], 0u);
        if (parts) {
            const uint32_t n = load_relaxed(&d.counters[C_NLIST]);
            if (d.pg.W == 1) closed += pull_close_wave<kCoopNE, kCoopNE>(d, par, wave0, nwaves, n, my_list);
            else pull_entries(d, tid, nthreads, n, par);
        }
        if (!grid_sync(d, epoch)) break;
        // close and push, for longer trajectories
        if (parts && d.pg.W > 1) {
            const uint32_t c = close_phase(d, par ^ 1, wave0, nwaves, my_list);  // same in every lane
            if (lane_id() == 0) closed += c;
            if (!grid_sync(d, epoch)) break;
        }
        ++r;
    }
    __syncthreads();
    if (closed) atomicAdd(&s_cnt, closed);  // LDS; per-lane counts
    __syncthreads();
    if (threadIdx.x == 0) slot_add(d, SL_PART_VISITS, s_cnt);
    if (tid == 0 && visits) atomicAdd(&d.stat64[S_TILE_VISITS], (unsigned long long)visits);
    if (tid == 0) {
        store_relaxed(&d.counters[C_ROUNDS], r - round0);
        store_relaxed(&d.counters[C_NWORK0 + (r & 1)], nwork);  // what remains (0 when converged)
    }
}

// ---- read-out ----

__device__ __forceinline__ bool gate_open(const ReadGate& gate) {
    return !gate.counters || gate.counters[C_ROUNDS] < gate.rounds || gate.counters[C_NWORK0 + gate.par] == 0u;
}

// Field labels -> canonical bit words ((t*Z + z)*Y + y)*X + x, with a member
// count.  When X is a multiple of 32 a canonical word is one tile word: a block
// stages up to 8 x-consecutive tiles in LDS (rows padded by one word against
// bank conflicts) and writes whole canonical rows.  Otherwise bit by bit.
template <int BT>
__global__ __launch_bounds__(256) void k_read_field_tiles(Dev d, uint32_t* __restrict__ out, int vec, ReadGate gate) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    constexpr int WPT = 64 * BT;
    __shared__ uint32_t sl[8 * (WPT + 1)];
    if (!gate_open(gate)) return;  // the same in every thread
    const Geom& g = d.g;
    const int ty = blockIdx.x, tz = blockIdx.y, tt = blockIdx.z;
    uint32_t cnt = 0;
    for (int tx0 = 0; tx0 < g.NXt; tx0 += 8) {
        const int ntx = min(8, g.NXt - tx0);
        const uint32_t tile0 = tile_of(g, tx0, ty, tz, tt);
        uint32_t act = 0;  // one bit per tile of this x-run; the same in every thread
        for (int k = 0; k < ntx; ++k) act |= (d.active[tile0 + k] != 0 ? 1u : 0u) << k;
        if (act) {
            const uint32_t* src = d.Lf + (size_t)tile0 * WPT;
            for (int i = threadIdx.x; i < ntx * WPT; i += 256) {
                const int txl = i / WPT, w = i - txl * WPT;
                sl[txl * (WPT + 1) + w] = (act >> txl) & 1u ? src[i] : 0u;
            }
            __syncthreads();
        }
        if (vec) {
            // a thread writes 4 x-consecutive words of one canonical row
            const int nq = ntx >> 2;
            for (int i = threadIdx.x; i < nq * WPT; i += 256) {
                const int qx = i % nq, w = i / nq;
                const int yl = w & 7, zl = (w >> 3) & 7, tl = w >> 6;
                const int y = ty * 8 + yl, z = tz * 8 + zl, t = tt * BT + tl;
                if (y < g.Y && z < g.Z && t < g.T) {
                    v4u v = {0u, 0u, 0u, 0u};
                    if (act) {
                        const uint32_t* r = sl + (4 * qx) * (WPT + 1) + w;
                        v = (v4u){r[0], r[WPT + 1], r[2 * (WPT + 1)], r[3 * (WPT + 1)]};
                        cnt += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
                    }
                    __builtin_nontemporal_store(
                        v, reinterpret_cast<v4u*>(out + ((size_t)(t * g.Z + z) * g.Y + y) * g.NXt + tx0 + 4 * qx));
                }
            }
        } else {
            for (int i = threadIdx.x; i < ntx * WPT; i += 256) {
                const int txl = i % ntx, w = i / ntx;
                const int yl = w & 7, zl = (w >> 3) & 7, tl = w >> 6;
                const int y = ty * 8 + yl, z = tz * 8 + zl, t = tt * BT + tl;
                if (y < g.Y && z < g.Z && t < g.T) {
                    const uint32_t v = act ? sl[txl * (WPT + 1) + w] : 0u;
                    out[((size_t)(t * g.Z + z) * g.Y + y) * g.NXt + tx0 + txl] = v;
                    cnt += __popc(v);
                }
            }
        }
        __syncthreads();
    }
    block_slot_sum(d, SL_MEMBERS_F, cnt);
}

__global__ __launch_bounds__(256) void k_read_field_bits(Dev d, uint32_t* __restrict__ out, ReadGate gate) {
    if (!gate_open(gate)) return;
    const Geom& g = d.g;
    const uint64_t V = (uint64_t)g.X * g.Y * g.Z * g.T;
    const uint64_t nw = (V + 31) >> 5;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t cnt = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nw; i += stride) {
        uint32_t w = 0;
        for (int k = 0; k < 32; ++k) {
            const uint64_t bi = i * 32 + k;
            if (bi >= V) break;
            const uint32_t x = (uint32_t)(bi % g.X);
            const uint64_t r = bi / g.X;
            const int y = r % g.Y;
            const uint64_t r2 = r / g.Y;
            const int z = r2 % g.Z, t = (int)(r2 / g.Z);
            const uint32_t b = bit_index(g, (int)x, y, z, t);
            if (d.active[b >> (5 + 6 + g.logBT)] && test_bit(d.Lf, b)) w |= 1u << k;
        }
        out[i] = w;
        cnt += __popc(w);
    }
    block_slot_sum(d, SL_MEMBERS_F, cnt);
}

// Particle labels -> uint8 [T][P].  Fast path (P a multiple of 16): a thread
// owns 16 consecutive particles and, label word by label word, writes their 16
// bytes of each step as one 16-byte store.
__global__ __launch_bounds__(256) void k_read_particles16(Dev d, uint8_t* __restrict__ out, ReadGate gate) {
    if (!gate_open(gate)) return;
    const PGeom& pg = d.pg;
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t p0 = q * 16;
    uint32_t cnt = 0;
    if (p0 < pg.P) {
        const uint4 fl = *reinterpret_cast<const uint4*>(d.pflag + p0);  // 16 candidate flags
        const uint32_t fw[4] = {fl.x, fl.y, fl.z, fl.w};
        const int nw = (pg.T + 63) >> 6;  // words holding real steps
        for (int w = 0; w < nw; ++w) {
            unsigned long long lw[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                lw[k] = (fw[k >> 2] >> (8 * (k & 3))) & 0xFFu ? d.Lp[(size_t)(p0 + k) * pg.W + w] : 0ull;
                cnt += __popcll(lw[k]);
            }
            const int tend = min(64, pg.T - w * 64);
            for (int t = 0; t < tend; ++t) {
                uint32_t v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    v[j] = (uint32_t)((lw[4 * j] >> t) & 1) | ((uint32_t)((lw[4 * j + 1] >> t) & 1) << 8) |
                           ((uint32_t)((lw[4 * j + 2] >> t) & 1) << 16) |
                           ((uint32_t)((lw[4 * j + 3] >> t) & 1) << 24);
                typedef unsigned int v4u __attribute__((ext_vector_type(4)));
                __builtin_nontemporal_store((v4u){v[0], v[1], v[2], v[3]},
                                            reinterpret_cast<v4u*>(out + (int64_t)(w * 64 + t) * pg.P + p0));
            }
        }
    }
    block_slot_sum(d, SL_MEMBERS_P, cnt);
}

// General particle read-out: a thread owns 4 consecutive particles.
__global__ __launch_bounds__(256) void k_read_particles(Dev d, uint8_t* __restrict__ out, ReadGate gate) {
    if (!gate_open(gate)) return;
    const PGeom& pg = d.pg;
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t p0 = q * 4;
    uint32_t cnt = 0;
    if (p0 < pg.P) {
        const int np = (int)min((int64_t)4, pg.P - p0);
        for (int w = 0; w < pg.W; ++w) {
            unsigned long long lw[4] = {0, 0, 0, 0};
            for (int k = 0; k < np; ++k) {
                lw[k] = d.pflag[p0 + k] ? d.Lp[(size_t)(p0 + k) * pg.W + w] : 0ull;
                cnt += __popcll(lw[k]);
            }
            const int tend = min(64, pg.T - w * 64);
            for (int tl = 0; tl < tend; ++tl) {
                const int64_t t = w * 64 + tl;
                uint8_t* o = out + t * pg.P + p0;
                for (int k = 0; k < np; ++k) o[k] = (uint8_t)((lw[k] >> tl) & 1);
            }
        }
    }
    block_slot_sum(d, SL_MEMBERS_P, cnt);
}

// Trajectory segments of the grown feature (Section 3.4): a member step stays
// when the same particle is a member at t - 1 or t + 1, so that only runs of
// two or more consecutive member steps are drawn.  On a label word L (bit t =
// step t) that is L & ((L << 1) | (L >> 1)), with the neighbouring words'
// edge bits carried in.  A thread owns 4 consecutive particles; out is uint8
// [T][P], written 4 bytes per step when the 4 are whole and aligned.
__global__ __launch_bounds__(256) void k_particle_segments(Dev d, uint8_t* __restrict__ out) {
    const PGeom& pg = d.pg;
    const int nw = (pg.T + 63) >> 6;  // words holding real steps
    const bool wide = (pg.P & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 3) == 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t p0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * 4; p0 < pg.P; p0 += stride) {
        const int np = (int)min((int64_t)4, pg.P - p0);
        bool cand[4];
        for (int k = 0; k < 4; ++k) cand[k] = k < np && d.pflag[p0 + k];
        auto word = [&](int k, int w) -> unsigned long long {
            if (w < 0 || w >= nw || !cand[k]) return 0ull;
            const int valid = min(64, pg.T - w * 64);
            const unsigned long long vm = valid >= 64 ? ~0ull : ((1ull << valid) - 1);
            return d.Lp[(size_t)(p0 + k) * pg.W + w] & vm;
        };
        for (int w = 0; w < nw; ++w) {
            unsigned long long keep[4];
            for (int k = 0; k < 4; ++k) {
                const unsigned long long L = word(k, w);
                const unsigned long long nb = (L << 1) | (word(k, w - 1) >> 63) | (L >> 1) |
                                              (word(k, w + 1) << 63);
                keep[k] = L & nb;
            }
            const int tend = min(64, pg.T - w * 64);
            for (int tl = 0; tl < tend; ++tl) {
                uint8_t* o = out + (int64_t)(w * 64 + tl) * pg.P + p0;
                if (wide) {
                    const uint32_t v = (uint32_t)((keep[0] >> tl) & 1) | ((uint32_t)((keep[1] >> tl) & 1) << 8) |
                                       ((uint32_t)((keep[2] >> tl) & 1) << 16) |
                                       ((uint32_t)((keep[3] >> tl) & 1) << 24);
                    *reinterpret_cast<uint32_t*>(o) = v;
                } else {
                    for (int k = 0; k < np; ++k) o[k] = (uint8_t)((keep[k] >> tl) & 1);
                }
            }
        }
    }
}

// Per-seed component ids, field part.  words: canonical member bits of a grow
// from one seed; seen: the members of the earlier seeds' grows.  A member no
// earlier grow reached takes `id` (seeds run in index order, so each node
// keeps the lowest index whose region holds it).  A thread owns whole words.
__global__ __launch_bounds__(256) void k_seed_ids_field(const uint32_t* __restrict__ words,
                                                        uint32_t* __restrict__ seen, uint64_t V, int32_t id,
                                                        int32_t* __restrict__ out) {
    const uint64_t nw = (V + 31) >> 5;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nw; i += stride) {
        const uint32_t w = words[i];
        if (!w) continue;
        const uint32_t s = seen[i];
        uint32_t n = w & ~s;
        if (!n) continue;
        seen[i] = s | n;
        while (n) {
            const uint64_t v = i * 32 + (uint64_t)(__ffs(n) - 1);
            n &= n - 1;
            if (v < V) out[v] = id;
        }
    }
}

// Per-seed component ids, particle part: the same over each particle's label
// words (seen: [P][ceil(T / 64)] words); out is int32 [T][P].
__global__ __launch_bounds__(256) void k_seed_ids_particles(Dev d, unsigned long long* __restrict__ seen,
                                                            int32_t id, int32_t* __restrict__ out) {
    const PGeom& pg = d.pg;
    const int nw = (pg.T + 63) >> 6;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < pg.P; p += stride) {
        if (!d.pflag[p]) continue;
        for (int w = 0; w < nw; ++w) {
            const int valid = min(64, pg.T - w * 64);
            const unsigned long long vm = valid >= 64 ? ~0ull : ((1ull << valid) - 1);
            const unsigned long long L = d.Lp[(size_t)p * pg.W + w] & vm;
            if (!L) continue;
            const unsigned long long s = seen[(size_t)p * nw + w];
            unsigned long long n = L & ~s;
            if (!n) continue;
            seen[(size_t)p * nw + w] = s | n;
            while (n) {
                const int64_t t = w * 64 + __builtin_ctzll(n);
                n &= n - 1;
                out[t * pg.P + p] = id;
            }
        }
    }
}

inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap) {
    uint64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

template <int BT>
bool coop_rounds(const Dev& d, uint32_t round0, uint32_t max_rounds, int device, hipStream_t s) {
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds<BT>, 256, 0) != hipSuccess ||
        per_cu <= 0)
        return false;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        ncu <= 0)
        return false;
    Dev dd = d;
    uint32_t r0 = round0, mr = max_rounds;
    void* args[] = {&dd, &r0, &mr};
    // Two blocks (8 waves) per CU: measured faster than four at 256^3 x 64,
    // where more blocks only add barrier arrivals.
    const dim3 grid((unsigned)(std::min(per_cu, 2) * ncu));
    return hipLaunchCooperativeKernel((const void*)k_rounds<BT>, grid, dim3(256), args, 0, s) ==
           hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

void launch_fold_slots(const Dev& d, int which, int dst, hipStream_t s, bool assign) {
    const FoldList f{1, {which, 0, 0, 0}, {dst, 0, 0, 0}, assign ? 1 : 0};
    hipLaunchKernelGGL(k_fold_slots, dim3(1), dim3(1024), 0, s, d, f);
}

const FoldList kGrowFold{3,
                         {SL_PART_VISITS, SL_ACTIVE, SL_TESTED, 0},
                         {S_PART_VISITS, S_ACTIVE_TILES, S_TILES_TESTED, 0},
                         0};

void launch_fold_grow_slots(const Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_fold_slots, dim3(1), dim3(1024), 0, s, d, kGrowFold);
}

void launch_chunk_end(const Dev& d, int par, uint32_t* snap, hipStream_t s) {
    hipLaunchKernelGGL(k_chunk_end, dim3(1), dim3(1024), 0, s, d, par, kGrowFold, snap);
}

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
}

void launch_reset(const Dev& d, hipStream_t s) {
    const uint64_t n = 2ull * d.g.NT + (uint64_t)(d.pg.P + 31) / 32;
    hipLaunchKernelGGL(k_reset, dim3(grid_for(n, 256, 2048)), dim3(256), 0, s, d);
}

void launch_bin_particles(const Geom& g, const PGeom& pg, const float* xyz, const float* attr,
                          uint32_t* bins, float* attr_t, hipStream_t s) {
    if (pg.P == 0) return;
    const unsigned nb = (unsigned)((pg.P + 63) / 64);
    hipLaunchKernelGGL(k_bin_particles, dim3(nb), dim3(256), 0, s, g, pg, xyz, attr, bins, attr_t);
}

void launch_summaries(const Geom& g, const float* field, float2* tsum, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_summaries, dim3(g.NT), dim3(256), 0, s, g, field, tsum);
}

void launch_particle_summaries(const PGeom& pg, const float* attr_t, float2* psum, hipStream_t s) {
    if (pg.P == 0) return;
    hipLaunchKernelGGL(k_particle_summaries, dim3(grid_for(pg.P, 256, 8192)), dim3(256), 0, s, pg,
                       attr_t, psum);
}

void launch_admit_field(const Dev& d, hipStream_t s) {
    if (d.admit_all) {
        hipLaunchKernelGGL(k_admit_field, dim3(d.g.NYt, d.g.NZt, d.g.T), dim3(256), 0, s, d);
        hipLaunchKernelGGL(k_count_active, dim3(grid_for(d.g.NT, 256, 1024)), dim3(256), 0, s, d);
    } else {
        // counts its active and tested tiles itself
        hipLaunchKernelGGL(k_tile_candidates, dim3(grid_for(d.g.NT, 256, 1024)), dim3(256), 0, s, d);
        hipLaunchKernelGGL(k_admit_tiles, dim3(grid_for(d.g.NT, 1, 8192)), dim3(256), 0, s, d);
    }
}

void launch_admit_particles(const Dev& d, hipStream_t s) {
    const PGeom& pg = d.pg;
    if (pg.P == 0) return;
    if (pg.Tpad >= 4) {
        const uint64_t n4 = ((uint64_t)pg.P * pg.Tpad) >> 2;
        (void)n4;
        hipLaunchKernelGGL(k_admit_particles, dim3(grid_for((uint64_t)pg.P, kAdmitChunk, 2048)), dim3(256), 0,
                           s, d);
    } else {
        hipLaunchKernelGGL(k_admit_particles_short, dim3(grid_for(pg.P, 256, 4096)), dim3(256), 0, s,
                           d);
        hipLaunchKernelGGL(k_couple, dim3(grid_for((uint64_t)pg.P * pg.W, 256, 8192)), dim3(256), 0,
                           s, d);
    }
}

void launch_seeds(const Dev& d, const int32_t* seeds, int64_t S, hipStream_t s) {
    if (S > 0)
        hipLaunchKernelGGL(k_seeds, dim3(grid_for(S, 256, 1u << 20)), dim3(256), 0, s, d, seeds, S);
}

void launch_work_total(const Dev& d, int par, hipStream_t s) {
    hipLaunchKernelGGL(k_work_total, dim3(1), dim3(64), 0, s, d, par);
}

void launch_round(const Dev& d, uint32_t round, hipStream_t s, hipEvent_t* ev) {
    if (ev) (void)hipEventRecord(ev[0], s);
    const int par = round & 1;
    // one wave per listed tile, up to 2048 waves (8 per CU); the list length
    // is on the device and longer lists are strided over the waves
    const uint64_t waves = d.g.NT < 2048u ? d.g.NT : 2048u;
    const unsigned blocks = grid_for(waves * 64, 256, 2048);
    switch (d.g.BT) {
        case 4: hipLaunchKernelGGL(k_round_sweep<4>, dim3(blocks), dim3(256), 0, s, d, par); break;
        case 8: hipLaunchKernelGGL(k_round_sweep<8>, dim3(blocks), dim3(256), 0, s, d, par); break;
        default: hipLaunchKernelGGL(k_round_sweep<16>, dim3(blocks), dim3(256), 0, s, d, par); break;
    }
    const uint64_t Q = (uint64_t)d.pg.P * d.pg.Tpad;
    if (ev) (void)hipEventRecord(ev[1], s);
    hipLaunchKernelGGL(k_round_pull, dim3(grid_for(Q / 4, 256, 2048)), dim3(256), 0, s, d, par);
    if (ev) (void)hipEventRecord(ev[2], s);
    // one thread per pdirty word (a wave takes 64), and enough to clear the tile flags
    const uint64_t nw32 = (uint64_t)(d.pg.P + 31) / 32;
    const uint64_t nclose = (uint64_t)d.g.NT > nw32 ? (uint64_t)d.g.NT : nw32;
    if (d.pg.W > 1)  // one label word per particle: closed inside the pull
        hipLaunchKernelGGL(k_round_close, dim3(grid_for(nclose, 256, 2048)), dim3(256), 0, s, d, par);
    if (ev) (void)hipEventRecord(ev[3], s);
}

bool launch_rounds_persistent(const Dev& d, uint32_t round0, uint32_t max_rounds, int device,
                              hipStream_t s) {
    switch (d.g.BT) {
        case 4: return coop_rounds<4>(d, round0, max_rounds, device, s);
        case 8: return coop_rounds<8>(d, round0, max_rounds, device, s);
        default: return coop_rounds<16>(d, round0, max_rounds, device, s);
    }
}

void launch_read_field(const Dev& d, uint32_t* out, hipStream_t s, const ReadGate& gate) {
    const Geom& g = d.g;
    if ((g.X & 31) == 0) {
        const dim3 grid(g.NYt, g.NZt, g.NTt);
        // 16-byte stores when every x-run of tiles is a multiple of 4 words
        const int vec = (g.NXt & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
        switch (g.BT) {
            case 4: hipLaunchKernelGGL(k_read_field_tiles<4>, grid, dim3(256), 0, s, d, out, vec, gate); break;
            case 8: hipLaunchKernelGGL(k_read_field_tiles<8>, grid, dim3(256), 0, s, d, out, vec, gate); break;
            default: hipLaunchKernelGGL(k_read_field_tiles<16>, grid, dim3(256), 0, s, d, out, vec, gate); break;
        }
        return;
    }
    const uint64_t V = (uint64_t)g.X * g.Y * g.Z * g.T;
    hipLaunchKernelGGL(k_read_field_bits, dim3(grid_for((V + 31) / 32, 256, 16384)), dim3(256), 0,
                       s, d, out, gate);
}

void launch_read_particles(const Dev& d, uint8_t* out, hipStream_t s, const ReadGate& gate) {
    const PGeom& pg = d.pg;
    if (pg.P == 0) return;
    if ((pg.P & 15) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
        hipLaunchKernelGGL(k_read_particles16, dim3(grid_for(pg.P / 16, 256, 1u << 20)), dim3(256),
                           0, s, d, out, gate);
        return;
    }
    hipLaunchKernelGGL(k_read_particles, dim3(grid_for((pg.P + 3) / 4, 256, 1u << 20)), dim3(256),
                       0, s, d, out, gate);
}

void launch_particle_segments(const Dev& d, uint8_t* out, hipStream_t s) {
    const PGeom& pg = d.pg;
    if (pg.P == 0 || pg.T == 0) return;
    hipLaunchKernelGGL(k_particle_segments, dim3(grid_for((pg.P + 3) / 4, 256, 1u << 16)), dim3(256), 0,
                       s, d, out);
}

void launch_seed_ids(const Dev& d, const uint32_t* words, uint32_t* seen_f, unsigned long long* seen_p,
                     int32_t id, int32_t* field_ids, int32_t* particle_ids, hipStream_t s) {
    const uint64_t V = (uint64_t)d.g.X * d.g.Y * d.g.Z * d.g.T;
    hipLaunchKernelGGL(k_seed_ids_field, dim3(grid_for((V + 31) / 32, 256, 16384)), dim3(256), 0, s, words,
                       seen_f, V, id, field_ids);
    if (particle_ids && d.pg.P > 0)
        hipLaunchKernelGGL(k_seed_ids_particles, dim3(grid_for((uint64_t)d.pg.P, 256, 16384)), dim3(256), 0, s,
                           d, seen_p, id, particle_ids);
}

void launch_priority_keys(const Dev& d, const float* logits, int bW, int bH, int bD, float thr, uint32_t* keys,
                          uint32_t* vals, uint32_t* count, hipStream_t s) {
    hipLaunchKernelGGL(k_priority_keys, dim3(grid_for(d.g.NT, 256, 1024)), dim3(256), 0, s, d, logits, bW, bH, bD,
                       thr, keys, vals, count);
}

void launch_priority_sweep(const Dev& d, const uint32_t* list, const uint32_t* count, int waves, hipStream_t s) {
    const unsigned blocks = (unsigned)std::max(1, waves / 4);
    switch (d.g.BT) {
        case 4: hipLaunchKernelGGL(k_priority_sweep<4>, dim3(blocks), dim3(256), 0, s, d, list, count, 0); break;
        case 8: hipLaunchKernelGGL(k_priority_sweep<8>, dim3(blocks), dim3(256), 0, s, d, list, count, 0); break;
        default: hipLaunchKernelGGL(k_priority_sweep<16>, dim3(blocks), dim3(256), 0, s, d, list, count, 0); break;
    }
}

void launch_verify_schedule(const Dev& d, int par, hipStream_t s) {
    hipLaunchKernelGGL(k_verify_schedule, dim3(grid_for(d.g.NT, 256, 1024)), dim3(256), 0, s, d, par);
}

void launch_jacobi(const Dev& d, const uint32_t* lf_cur, const unsigned long long* lp_cur, uint32_t* lf_nxt,
                   unsigned long long* lp_nxt, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_field, dim3(grid_for(d.g.nwords, 256, 16384)), dim3(256), 0, s, d, lf_cur, lf_nxt);
    if (d.pg.P > 0)
        hipLaunchKernelGGL(k_jacobi_particles, dim3(grid_for((uint64_t)d.pg.P * d.pg.Tpad, 256, 16384)), dim3(256), 0,
                           s, d, lf_cur, lp_cur, lf_nxt, lp_nxt);
}

}  // namespace mf4d
