// Batched growing: up to 256 queries (each its own seeds and criteria) as the
// bit-planes of one 256-bit label per node, grown together in one pass over
// the data.  Query q lives in bit (q & 31) of word (q >> 5) of every node.
//
// Admissibility of a value v for all queries at once: with the lower bounds
// sorted ascending, {q : lo_q <= v} is the first rank_lo(v) queries of that
// order, a prefix mask read from a table; likewise for the upper bounds sorted
// descending.  The node's 256-bit mask is the AND of the two table rows.
//
// The two ranks of every voxel-step and particle-step (rank_lo | rank_hi <<
// 16) are computed once per grow, when its admissibility is first read, and
// kept: sweeps, pulls and closes rebuild a node's 256-bit mask from them with
// two rows of the prefix tables (staged in LDS), no search.
//
// Field labels are grown in place in the caller's [V][8] output (canonical
// voxel order); particle labels in the caller's [T][P][8] output.  Work is
// organised in 4D tiles of 512 voxel-steps (a power-of-two extent per axis,
// chosen per context, e.g. 8 x 4 x 4 x 4), one thread per voxel-step, with
// the round protocol of the single-query grower: sweep, pull, close/push,
// double-buffered work lists by round parity.
#include "mf4d_internal.h"
#include "batched.h"

namespace mf4d {

namespace {

constexpr int kWave = 64;
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

struct Mask8 {
    uint32_t w[8];
};

// #{i : s[i] <= v} for s ascending (n <= 256); NaN v gives 0.
// The predicate holds on a prefix of s: its length by halving steps of
// fixed sizes (every lane takes the same steps: no divergence, one LDS read
// each).
__device__ __forceinline__ int rank_le(const float* s, int n, float v) {
    if (n <= 0) return 0;
    int pos = 0;
    for (int step = 1 << (31 - __clz(n)); step > 0; step >>= 1)
        if (pos + step <= n && s[pos + step - 1] <= v) pos += step;
    return pos;
}
// #{i : s[i] >= v} for s descending.
__device__ __forceinline__ int rank_ge(const float* s, int n, float v) {
    if (n <= 0) return 0;
    int pos = 0;
    for (int step = 1 << (31 - __clz(n)); step > 0; step >>= 1)
        if (pos + step <= n && s[pos + step - 1] >= v) pos += step;
    return pos;
}

// Tables: sorted bounds and prefix masks, for one sample type.
struct BandTables {
    const float* lo_sorted;  // ascending, Q
    const float* hi_sorted;  // descending, Q
    const uint32_t* lo_mask; // [Q+1][8]
    const uint32_t* hi_mask; // [Q+1][8]
};

__device__ __forceinline__ Mask8 band_mask(const BandTables& tb, int Q, float v) {
    const int rl = rank_le(tb.lo_sorted, Q, v);
    const int rh = rank_ge(tb.hi_sorted, Q, v);
    Mask8 m;
#pragma unroll
    for (int k = 0; k < 8; ++k) m.w[k] = tb.lo_mask[rl * 8 + k] & tb.hi_mask[rh * 8 + k];
    return m;
}

// Prefix-mask tables of one sample type staged in LDS: lo rows then hi rows,
// [257][8] words each.
constexpr int kLdsTab = 2 * 257 * 8;

__device__ __forceinline__ void stage_tables(const DevB& d, int type, uint32_t* s_tab) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(d.tab + 1024) + (size_t)type * 2 * 257 * 8;
    for (int i = threadIdx.x; i < kLdsTab; i += blockDim.x) s_tab[i] = src[i];
}

// Word k of the mask of a node with packed ranks r, from staged tables.
__device__ __forceinline__ uint32_t rank_word(const uint32_t* s_tab, uint32_t r, int k) {
    return s_tab[(r & 0xFFFFu) * 8 + k] & s_tab[257 * 8 + (r >> 16) * 8 + k];
}

__device__ __forceinline__ BandTables field_tables(const DevB& d) {
    return BandTables{d.tab, d.tab + 256, reinterpret_cast<const uint32_t*>(d.tab + 1024),
                      reinterpret_cast<const uint32_t*>(d.tab + 1024) + 257 * 8};
}

__device__ __forceinline__ uint32_t btile_of(const DevB& d, int x, int y, int z, int t) {
    return ((uint32_t)((t >> d.lt) * d.NZb + (z >> d.lz)) * d.NYb + (y >> d.ly)) * d.NXb + (x >> d.lx);
}

__device__ __forceinline__ void btile_coords(const DevB& d, uint32_t tile, int& bx, int& by, int& bz,
                                             int& bt) {
    bx = tile % d.NXb;
    tile /= d.NXb;
    by = tile % d.NYb;
    tile /= d.NYb;
    bz = tile % d.NZb;
    bt = tile / d.NZb;
}

__device__ __forceinline__ uint64_t vindex(const DevB& d, int x, int y, int z, int t) {
    return (((uint64_t)t * d.Z + z) * d.Y + y) * d.X + x;
}

// Canonical voxel of a tile-layout bit position (the single-query binning).
__device__ __forceinline__ void bit_to_xyzt(const Geom& g, uint32_t b, int& x, int& y, int& z,
                                            int& t) {
    const uint32_t word = b >> 5;
    const uint32_t tile = word >> (6 + g.logBT);
    const uint32_t wi = word & (g.WPT - 1);
    uint32_t r = tile;
    const int tx = r % g.NXt;
    r /= g.NXt;
    const int ty = r % g.NYt;
    r /= g.NYt;
    const int tz = r % g.NZt;
    const int tt = r / g.NZt;
    x = tx * 32 + (b & 31);
    y = ty * 8 + (wi & 7);
    z = tz * 8 + ((wi >> 3) & 7);
    t = (tt << g.logBT) + (wi >> 6);
}

// Scheduling flags a tile for the round of parity `par` with a plain store
// (no round trip to wait for); kb_compact turns the flags into that round's
// work list, dropping tiles without an admissible node.
__device__ __forceinline__ void bschedule(const DevB& d, uint32_t tile, int par) {
    d.dirty[par * d.NTB + tile] = 1u;
}

template <int N>
__device__ __forceinline__ void bschedule_n(const DevB& d, const uint32_t (&tiles)[N], int par) {
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (tiles[i] != ~0u) bschedule(d, tiles[i], par);
}

// The voxel's tile (flagged for the pull) and the tiles whose face it
// touches, at most one per axis: slots 0 (own) and 1..4 of nb (~0u: none).
__device__ __forceinline__ void voxel_targets(const DevB& d, int x, int y, int z, int t, int par,
                                              uint32_t* nb) {
    const uint32_t tile = btile_of(d, x, y, z, t);
    d.chg[par * d.NTB + tile] = 1;
    const uint32_t sy = d.NXb, sz = d.NXb * d.NYb, st = sz * d.NZb;
    const int mx = (1 << d.lx) - 1, my = (1 << d.ly) - 1, mz = (1 << d.lz) - 1, mt = (1 << d.lt) - 1;
    nb[0] = tile;
    nb[1] = nb[2] = nb[3] = nb[4] = ~0u;
    if ((x & mx) == 0 && x > 0) nb[1] = tile - 1;
    else if ((x & mx) == mx && x + 1 < d.X) nb[1] = tile + 1;
    if ((y & my) == 0 && y > 0) nb[2] = tile - sy;
    else if ((y & my) == my && y + 1 < d.Y) nb[2] = tile + sy;
    if ((z & mz) == 0 && z > 0) nb[3] = tile - sz;
    else if ((z & mz) == mz && z + 1 < d.Z) nb[3] = tile + sz;
    if ((t & mt) == 0 && t > 0) nb[4] = tile - st;
    else if ((t & mt) == mt && t + 1 < d.T) nb[4] = tile + st;
}

__device__ __forceinline__ void bmark_voxel(const DevB& d, int x, int y, int z, int t, int par) {
    uint32_t nb[5];
    voxel_targets(d, x, y, z, t, par, nb);
    bschedule_n<5>(d, nb, par);
}

// N voxels (bit positions, kNoVoxel: none) marked together.
template <int N>
__device__ __forceinline__ void bmark_voxels_n(const DevB& d, const uint32_t (&b)[N], int par) {
    uint32_t nb[5 * N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < 5; ++j) nb[5 * i + j] = ~0u;
        if (b[i] != kNoVoxel) {
            int x, y, z, t;
            bit_to_xyzt(d.g, b[i], x, y, z, t);
            voxel_targets(d, x, y, z, t, par, nb + 5 * i);
        }
    }
    bschedule_n<5 * N>(d, nb, par);
}

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_tmp,
                                                        uint32_t& total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_tmp[wave] = x;
    __syncthreads();
    uint32_t wbase = 0;
    total = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) wbase += s_tmp[w];
        total += s_tmp[w];
    }
    __syncthreads();
    return wbase + x - v;
}

__device__ __forceinline__ uint32_t block_append(uint32_t n, uint32_t* counter, uint32_t* s_tmp) {
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(n, s_tmp, total);
    if (threadIdx.x == 0) s_tmp[16] = total ? atomicAdd(counter, total) : 0u;
    __syncthreads();
    const uint32_t base = s_tmp[16];
    __syncthreads();
    return base + ex;
}

// ---------------------------------------------------------------------------

// The sorted bounds of one sample type staged in LDS (lo ascending, then hi
// descending, 256 each), for the rank searches of a whole block.
__device__ __forceinline__ void stage_bounds(const DevB& d, int type, float* s_b) {
    for (int i = threadIdx.x; i < 512; i += blockDim.x) s_b[i] = d.tab[512 * type + i];
}

// Clear both output planes, record every voxel-step's ranks, mark tiles that
// hold a node admissible for some query.  One thread per voxel-step
// (canonical order), a grid-stride loop.
__global__ __launch_bounds__(256) void kb_admit_field(DevB d) {
    __shared__ float s_b[512];
    stage_bounds(d, 0, s_b);
    __syncthreads();
    const uint32_t* ftab = reinterpret_cast<const uint32_t*>(d.tab + 1024);
    const uint64_t V = (uint64_t)d.X * d.Y * d.Z * d.T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // four voxel-steps per thread and pass (stride apart, so each load and
    // store instruction stays coalesced): their rank searches interleave
    constexpr int kU = 4;
    for (uint64_t v0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v0 < V; v0 += kU * stride) {
        float f[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint64_t v = v0 + u * stride;
            f[u] = v < V ? __builtin_nontemporal_load(d.field + v) : 0.0f;
        }
        uint32_t r[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
            r[u] = (uint32_t)rank_le(s_b, d.Q, f[u]) | ((uint32_t)rank_ge(s_b + 256, d.Q, f[u]) << 16);
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint64_t v = v0 + u * stride;
            if (v >= V) continue;
            d.vrank[v] = r[u];
            uint4* o = reinterpret_cast<uint4*>(d.fplanes + v * 8);
            o[0] = make_uint4(0, 0, 0, 0);
            o[1] = make_uint4(0, 0, 0, 0);
            uint32_t any = 0;
            if ((r[u] & 0xFFFFu) && (r[u] >> 16)) {
#pragma unroll
                for (int k = 0; k < 8; ++k) any |= rank_word(ftab, r[u], k);
            }
            if (any) {
                const int x = (int)(v % d.X);
                const uint64_t q = v / d.X;
                const int y = (int)(q % d.Y);
                const uint64_t q2 = q / d.Y;
                const int z = (int)(q2 % d.Z), t = (int)(q2 / d.Z);
                d.active[btile_of(d, x, y, z, t)] = 1;
            }
        }
    }
}

// Clear the particle planes and list the coupled steps: admissible for some
// query and lying in a voxel, as (flat step index, canonical voxel index).
__global__ __launch_bounds__(256) void kb_admit_particles(DevB d) {
    __shared__ uint32_t s_tmp[20];
    __shared__ float s_b[512];
    stage_bounds(d, 1, s_b);
    __syncthreads();
    const uint32_t* ptab = reinterpret_cast<const uint32_t*>(d.tab + 1024) + 2 * 257 * 8;
    const uint64_t n = (uint64_t)d.P * d.Tpad;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t np = (uint64_t)d.Tp * d.P * 2;  // uint4 per particle-step: 2
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < np; i += stride)
        reinterpret_cast<uint4*>(d.pplanes)[i] = make_uint4(0, 0, 0, 0);
    for (uint64_t b0 = blockIdx.x * (uint64_t)blockDim.x; b0 < n; b0 += stride) {
        const uint64_t e = b0 + threadIdx.x;
        bool c = false;
        uint32_t vox = 0;
        if (e < n) {
            const float a = d.attr_t[e];
            const uint32_t r = (uint32_t)rank_le(s_b, d.Q, a) | ((uint32_t)rank_ge(s_b + 256, d.Q, a) << 16);
            d.prank[e] = r;
            uint32_t any = 0;
            if ((r & 0xFFFFu) && (r >> 16)) {
#pragma unroll
                for (int k = 0; k < 8; ++k) any |= rank_word(ptab, r, k);
            }
            const uint32_t b = d.bins[e];
            if (any && b != kNoVoxel) {
                int x, y, z, t;
                bit_to_xyzt(d.g, b, x, y, z, t);
                vox = (uint32_t)vindex(d, x, y, z, t);
                c = true;
            }
        }
        const uint32_t k = block_append(c ? 1u : 0u, &d.counters[BC_NLIST], s_tmp);
        if (c) d.clist[k] = make_uint2((uint32_t)e, vox);
    }
}

__global__ void kb_seeds(DevB d, const int32_t* __restrict__ seeds, int64_t S) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= S) return;
    const int32_t* s = seeds + 5 * i;
    const int x = s[0], y = s[1], z = s[2], t = s[3], q = s[4];
    const uint64_t v = vindex(d, x, y, z, t);
    const Mask8 m = band_mask(field_tables(d), d.Q, d.field[v]);
    const uint32_t bit = 1u << (q & 31);
    if (m.w[q >> 5] & bit) {
        if (!(atomicOr(&d.fplanes[v * 8 + (q >> 5)], bit) & bit)) bmark_voxel(d, x, y, z, t, 0);
    } else {
        atomicAdd(&d.counters[BC_DROPPED], 1u);
    }
}

// Lane moves within a row of 16 lanes (DPP): lane i receives lane i - N
// (shr) or i + N (shl) of its row; a lane whose source lies outside the row
// receives 0.  Register-only: no LDS traffic.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_row(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
constexpr int kDppRowShr1 = 0x111, kDppRowShr4 = 0x114, kDppRowShl1 = 0x101, kDppRowShl4 = 0x104;

// Sweep one tile (block of 512 threads, one voxel-step each) to a local fixed
// point: Jacobi steps through LDS over the 8 in-tile neighbours, the out-of-
// tile neighbours entering as fixed halos.  Tiles of 4 x 4 x 4 x 8 take a
// faster route: a wave holds one 4 x 4 x 4 cube at one t (a row of 16 lanes
// is one z-plane), so x and y neighbours are DPP row moves and z neighbours
// lane permutes; each wave runs its cube to a fixed point with the t
// neighbours held fixed, and only the t neighbours go through LDS, once per
// block-wide pass.
template <bool kCube>
__device__ void bsweep_tile(const DevB& d, uint32_t tile, int par, uint32_t* s_lab,
                            uint32_t* s_flags, const uint32_t* s_ftab) {
    int bx, by, bz, bt;
    btile_coords(d, tile, bx, by, bz, bt);
    const int tid = threadIdx.x;
    const int mx = (1 << d.lx) - 1, my = (1 << d.ly) - 1, mz = (1 << d.lz) - 1, mt = (1 << d.lt) - 1;
    const int sxl = 1, syl = 1 << d.lx, szl = 1 << (d.lx + d.ly), stl = 1 << (d.lx + d.ly + d.lz);
    const int xl = tid & mx, yl = (tid >> d.lx) & my, zl = (tid >> (d.lx + d.ly)) & mz,
              tl = tid >> (d.lx + d.ly + d.lz);
    const int x = (bx << d.lx) + xl, y = (by << d.ly) + yl, z = (bz << d.lz) + zl, t = (bt << d.lt) + tl;
    const bool in = x < d.X && y < d.Y && z < d.Z && t < d.T;
    if (tid == 0) {
        s_flags[0] = 0;
        s_flags[1] = 0;
        s_flags[2] = 0;
    }
    // a: the admissible queries per word; the cube route recomputes them
    // from the node's ranks where it needs them (fewer registers, more
    // blocks per CU)
    uint32_t a[8], l[8], h[8];
    uint32_t rv = 0;  // ranks 0: no query admits the node
    const uint64_t v = in ? vindex(d, x, y, z, t) : 0;
    if (in) {
        rv = d.vrank[v];
        const uint4* lp = reinterpret_cast<const uint4*>(d.fplanes + v * 8);
        const uint4 l01 = lp[0], l23 = lp[1];
        l[0] = l01.x; l[1] = l01.y; l[2] = l01.z; l[3] = l01.w;
        l[4] = l23.x; l[5] = l23.y; l[6] = l23.z; l[7] = l23.w;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = kCube ? 0u : rank_word(s_ftab, rv, k);
            h[k] = 0;
        }
        // halos: neighbours outside the tile (inside the grid), each load
        // issued on its own condition (no indexed list: it would live in
        // scratch memory)
        const uint64_t sx = 1, sy = d.X, sz = (uint64_t)d.X * d.Y, st = sz * d.Z;
        auto halo = [&](bool has, uint64_t nv) {
            if (!has) return;
            const uint4* hp = reinterpret_cast<const uint4*>(d.fplanes + nv * 8);
            const uint4 h01 = hp[0], h23 = hp[1];
            h[0] |= h01.x; h[1] |= h01.y; h[2] |= h01.z; h[3] |= h01.w;
            h[4] |= h23.x; h[5] |= h23.y; h[6] |= h23.z; h[7] |= h23.w;
        };
        halo(xl == 0 && x > 0, v - sx);
        halo(xl == mx && x + 1 < d.X, v + sx);
        halo(yl == 0 && y > 0, v - sy);
        halo(yl == my && y + 1 < d.Y, v + sy);
        halo(zl == 0 && z > 0, v - sz);
        halo(zl == mz && z + 1 < d.Z, v + sz);
        halo(tl == 0 && t > 0, v - st);
        halo(tl == mt && t + 1 < d.T, v + st);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = l[k] = h[k] = 0;
    }
    uint32_t grown = 0;  // some word of this node gained bits in this visit
    // in-tile neighbour thread ids (or -1)
    const int nx0 = xl > 0 ? tid - sxl : -1, nx1 = xl < mx ? tid + sxl : -1;
    const int ny0 = yl > 0 ? tid - syl : -1, ny1 = yl < my ? tid + syl : -1;
    const int nz0 = zl > 0 ? tid - szl : -1, nz1 = zl < mz ? tid + szl : -1;
    const int nt0 = tl > 0 ? tid - stl : -1, nt1 = tl < mt ? tid + stl : -1;
    const int nbr[8] = {nx0, nx1, ny0, ny1, nz0, nz1, nt0, nt1};
    // Words that can change in this visit: some voxel has room to grow in the
    // word (admissible, not a member) and some voxel or halo holds members of
    // it.  Most tiles carry few of the 8 words' queries; the others are left
    // out of the Jacobi steps (block-uniform).
    {
        uint32_t room = 0, src = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            room |= ((kCube ? rank_word(s_ftab, rv, k) : a[k]) & ~l[k]) ? 1u << k : 0u;
            src |= (l[k] | h[k]) ? 1u << k : 0u;
        }
        __syncthreads();  // the flags were cleared
        if (room) atomicOr(&s_flags[1], room);
        if (src) atomicOr(&s_flags[2], src);
        __syncthreads();
    }
    const uint32_t need = s_flags[1] & s_flags[2];
    // Gauss-Seidel through LDS: the needed words go to LDS once; then each
    // iteration a voxel with room to grow in a word (admissible for a query
    // it is not a member of) ORs its neighbours' current words into it and
    // writes the word back at once if it grew, so a change can travel on
    // within the same iteration (to waves that read after it).  A saturated
    // word cannot change and loads nothing.  Reads racing with writes only
    // see fewer bits (labels only grow); an iteration in which no voxel
    // changed read final values everywhere, which is the local fixed point.
    // The eight words are handled one by one (the register arrays stay in
    // registers only with constant indices).
#define MF4D_STORE_WORD(k) \
    if ((need >> (k)) & 1u) s_lab[(k) * 512 + tid] = l[k];
#define MF4D_STEP_WORD(k)                                                   \
    if (((need >> (k)) & 1u) && (a[k] & ~l[k])) {                          \
        uint32_t nbv = l[k] | h[k];                                         \
        _Pragma("unroll") for (int j = 0; j < 8; ++j)                       \
            if (nbr[j] >= 0) nbv |= s_lab[(k) * 512 + nbr[j]];              \
        const uint32_t sv = nbv & a[k];                                     \
        if (sv != l[k]) {                                                   \
            diff = 1u;                                                      \
            grown = 1u;                                                     \
            l[k] = sv;                                                      \
            s_lab[(k) * 512 + tid] = sv;                                    \
        }                                                                   \
    }
    // The cube route: word k's in-wave fixed point with its t neighbours'
    // words (read from LDS) and the halos held fixed.  A lane gains only
    // bits admissible for it; labels only grow, so the loop ends.
#define MF4D_CUBE_WORD(k)                                                       \
    if ((need >> (k)) & 1u) {                                                  \
        uint32_t fx = h[k];                                                    \
        if (nt0 >= 0) fx |= s_lab[(k) * 512 + nt0];                            \
        if (nt1 >= 0) fx |= s_lab[(k) * 512 + nt1];                            \
        const uint32_t ak = rank_word(s_ftab, rv, k);                          \
        uint32_t cur = l[k];                                                   \
        while (true) {                                                         \
            const uint32_t xm = dpp_row<kDppRowShr1>(cur);                     \
            const uint32_t xp = dpp_row<kDppRowShl1>(cur);                     \
            const uint32_t ym = dpp_row<kDppRowShr4>(cur);                     \
            const uint32_t yp = dpp_row<kDppRowShl4>(cur);                     \
            const uint32_t zm = (uint32_t)__shfl((int)cur, (lane - 16) & 63);   \
            const uint32_t zp = (uint32_t)__shfl((int)cur, (lane + 16) & 63);   \
            uint32_t nb = fx;                                                  \
            if (xl > 0) nb |= xm;                                              \
            if (xl < 3) nb |= xp;                                              \
            if (yl > 0) nb |= ym;                                              \
            if (yl < 3) nb |= yp;                                              \
            if (zl > 0) nb |= zm;                                              \
            if (zl < 3) nb |= zp;                                              \
            const uint32_t nv = cur | (nb & ak);                               \
            const bool grew = nv != cur;                                       \
            cur = nv;                                                          \
            if (__ballot(grew) == 0) break;                                    \
        }                                                                      \
        if (cur != l[k]) {                                                     \
            diff = 1u;                                                         \
            grown = 1u;                                                        \
            l[k] = cur;                                                        \
        }                                                                      \
    }
    if (kCube && need) {
        const int lane = tid & 63;
        while (true) {
            MF4D_STORE_WORD(0) MF4D_STORE_WORD(1) MF4D_STORE_WORD(2) MF4D_STORE_WORD(3)
            MF4D_STORE_WORD(4) MF4D_STORE_WORD(5) MF4D_STORE_WORD(6) MF4D_STORE_WORD(7)
            __syncthreads();
            uint32_t diff = 0;
            MF4D_CUBE_WORD(0) MF4D_CUBE_WORD(1) MF4D_CUBE_WORD(2) MF4D_CUBE_WORD(3)
            MF4D_CUBE_WORD(4) MF4D_CUBE_WORD(5) MF4D_CUBE_WORD(6) MF4D_CUBE_WORD(7)
            // every wave has read its t neighbours before the next pass
            // stores; a pass with no change anywhere is the fixed point
            if (!__syncthreads_or(diff != 0)) break;
        }
    } else if (need) {
        MF4D_STORE_WORD(0) MF4D_STORE_WORD(1) MF4D_STORE_WORD(2) MF4D_STORE_WORD(3)
        MF4D_STORE_WORD(4) MF4D_STORE_WORD(5) MF4D_STORE_WORD(6) MF4D_STORE_WORD(7)
        __syncthreads();
        while (true) {
            uint32_t diff = 0;
            MF4D_STEP_WORD(0) MF4D_STEP_WORD(1) MF4D_STEP_WORD(2) MF4D_STEP_WORD(3)
            MF4D_STEP_WORD(4) MF4D_STEP_WORD(5) MF4D_STEP_WORD(6) MF4D_STEP_WORD(7)
            if (!__syncthreads_or(diff != 0)) break;
        }
    }
#undef MF4D_CUBE_WORD
#undef MF4D_STORE_WORD
#undef MF4D_STEP_WORD
    uint32_t any = 0;
    if (in) {
        any = grown;
        // a tile is swept by one block per phase and nothing else writes its
        // nodes meanwhile (seeds and pushes come in other phases): the node's
        // 32 bytes go back with two plain stores
        if (any) {
            uint4* lp = reinterpret_cast<uint4*>(d.fplanes + v * 8);
            lp[0] = make_uint4(l[0], l[1], l[2], l[3]);
            lp[1] = make_uint4(l[4], l[5], l[6], l[7]);
        }
    }
    if (any) {
        uint32_t faces = 1u << 8;  // bit 8: tile changed
        if (xl == 0) faces |= 1u << 0;
        if (xl == mx) faces |= 1u << 1;
        if (yl == 0) faces |= 1u << 2;
        if (yl == my) faces |= 1u << 3;
        if (zl == 0) faces |= 1u << 4;
        if (zl == mz) faces |= 1u << 5;
        if (tl == 0) faces |= 1u << 6;
        if (tl == mt) faces |= 1u << 7;
        atomicOr(&s_flags[0], faces);
    }
    __syncthreads();
    // lanes 0..7 of the first wave flag the tiles across the eight faces
    // that gained bits
    const uint32_t f = s_flags[0];
    if (f && tid < 8) {
        if (tid == 0) d.chg[par * d.NTB + tile] = 1;
        const uint32_t sy = d.NXb, sz = d.NXb * d.NYb, st = sz * d.NZb;
        uint32_t nb[1] = {~0u};
        if ((f >> tid) & 1u) {
            switch (tid) {
                case 0: if (bx > 0) nb[0] = tile - 1; break;
                case 1: if (bx + 1 < d.NXb) nb[0] = tile + 1; break;
                case 2: if (by > 0) nb[0] = tile - sy; break;
                case 3: if (by + 1 < d.NYb) nb[0] = tile + sy; break;
                case 4: if (bz > 0) nb[0] = tile - sz; break;
                case 5: if (bz + 1 < d.NZb) nb[0] = tile + sz; break;
                case 6: if (bt > 0) nb[0] = tile - st; break;
                default: if (bt + 1 < d.NTb) nb[0] = tile + st; break;
            }
        }
        bschedule_n<1>(d, nb, par ^ 1);
    }
    __syncthreads();
}

// A round's sweep.  Rounds are queued ahead of the host: a round whose work
// list is empty does nothing (its sweep records that for the round's pull and
// close), and BC_ROUNDS counts the rounds that had work.
// kCube: tiles of 4 x 4 x 4 x 8 (the cube route of bsweep_tile).
template <bool kCube>
__global__ __launch_bounds__(512) void kb_sweep(DevB d, int par) {
    __shared__ uint32_t s_lab[8 * 512];
    __shared__ uint32_t s_flags[4];
    __shared__ uint32_t s_ftab[kLdsTab];
    __shared__ uint32_t s_pref[kBSubs + 1];  // sub-list prefix sums
    if (threadIdx.x < kBSubs) {
        // the first wave scans the sub-list lengths
        const uint32_t c = d.wcnt[((uint32_t)par * kBSubs + threadIdx.x) * kBCntStride];
        uint32_t x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if ((int)threadIdx.x >= o) x += y;
        }
        s_pref[threadIdx.x + 1] = x;
        if (threadIdx.x == 0) s_pref[0] = 0;
    }
    __syncthreads();
    const uint32_t nwork = s_pref[kBSubs];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.counters[BC_NDIRTYP] = 0;
        d.counters[BC_RACT] = nwork ? 1u : 0u;
        if (nwork) d.counters[BC_ROUNDS] += 1u;
    }
    if (blockIdx.x >= nwork) return;  // block-uniform
    stage_tables(d, 0, s_ftab);
    __syncthreads();
    uint32_t visits = 0;
    for (uint32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        // the sub-list holding flat item w: the last j with s_pref[j] <= w
        int lo = 0, hi = kBSubs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_pref[mid] <= w) lo = mid; else hi = mid;
        }
        const uint32_t tile = d.work[((size_t)par * kBSubs + lo) * d.WCAPB + (w - s_pref[lo])];
        bsweep_tile<kCube>(d, tile, par, s_lab, s_flags, s_ftab);
        ++visits;
    }
    if (threadIdx.x == 0 && visits) atomicAdd(&d.stat64[S_TILE_VISITS], (unsigned long long)visits);
}

// Pull: a coupled step gains the queries for which its voxel is a member and
// it is admissible.
__global__ __launch_bounds__(256) void kb_pull(DevB d, int par) {
    __shared__ uint32_t s_tmp[20];
    if (!d.counters[BC_RACT]) return;
    const uint32_t* ptab = reinterpret_cast<const uint32_t*>(d.tab + 1024) + 2 * 257 * 8;
    const uint32_t n = d.counters[BC_NLIST];
    for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < n; b0 += gridDim.x * blockDim.x) {
        const uint32_t i = b0 + threadIdx.x;
        bool first = false;
        uint32_t p = 0;
        if (i < n) {
            const uint2 ent = d.clist[i];
            const uint32_t vox = ent.y;
            int x = (int)(vox % d.X);
            uint32_t r = vox / d.X;
            const int y = r % d.Y;
            r /= d.Y;
            const int z = r % d.Z, t = r / d.Z;
            if (d.chg[par * d.NTB + btile_of(d, x, y, z, t)]) {
                p = ent.x / (uint32_t)d.Tpad;
                const uint32_t ts = ent.x - p * (uint32_t)d.Tpad;
                const uint32_t* lf = d.fplanes + (uint64_t)vox * 8;
                uint32_t* lp = d.pplanes + ((uint64_t)ts * d.P + p) * 8;
                bool any = false;
                bool got = false;
                Mask8 m;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    m.w[k] = lf[k] & ~lp[k];
                    any |= m.w[k] != 0;
                }
                if (any) {
                    const uint32_t rp = d.prank[ent.x];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const uint32_t nw = m.w[k] & rank_word(ptab, rp, k);
                        if (nw && (~atomicOr(&lp[k], nw) & nw)) got = true;
                    }
                }
                if (got) {
                    const uint32_t pb = 1u << (p & 31);
                    first = !(atomicOr(&d.pdirty[p >> 5], pb) & pb);
                }
            }
        }
        const uint32_t k = block_append(first ? 1u : 0u, &d.counters[BC_NDIRTYP], s_tmp);
        if (first) d.dlist[k] = p;
    }
}

// Close and push the dirty particles for every query plane, eight lanes per
// particle: lane k of a group of eight carries word k (queries 32k .. 32k +
// 31) along the particle's steps.  A forward and a backward pass spread the
// members over admissible runs (the forward pass alone with forward-only
// coupling); a step that gains queries pushes them into its voxel where the
// voxel is admissible, and one lane of the group marks the voxel when any
// word of it was gained.  The steps go in chunks of kChunk: every load of a
// chunk (labels, ranks, bins; then the pushed voxels' ranks; then their
// atomics) is issued together, so a chunk costs a few round trips instead of
// a few per step.  Every lane runs every chunk (ballots).
constexpr int kChunk = 16;

// A whole trajectory of up to kWhole steps closed in registers (lane k of the
// particle's group of eight carries word k): every step's label, ranks and bin
// are loaded at once (one round trip), the forward and the backward pass run
// on them, and the new bits are written and pushed in two halves, each half's
// loads and atomics issued together.  Every lane of the wave calls it.
constexpr int kWhole = 32;
__device__ __forceinline__ void close_whole(const DevB& d, uint32_t p, bool valid, int k, int grp, int npar,
                                            const uint32_t* s_ptab, const uint32_t* s_ftab) {
    const int Tp = d.Tp;
    uint32_t lab[kWhole], cur[kWhole], adm[kWhole], bin[kWhole];
#pragma unroll
    for (int j = 0; j < kWhole; ++j) {
        cur[j] = 0;
        adm[j] = 0;
        bin[j] = kNoVoxel;
        if (valid && j < Tp) {
            cur[j] = d.pplanes[((uint64_t)j * d.P + p) * 8 + k];
            adm[j] = d.prank[(uint64_t)p * d.Tpad + j];
            bin[j] = d.bins[(uint64_t)p * d.Tpad + j];
        }
    }
#pragma unroll
    for (int j = 0; j < kWhole; ++j) adm[j] = j < Tp && valid ? rank_word(s_ptab, adm[j], k) : 0u;
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < kWhole; ++j) {
        lab[j] = cur[j] | (carry & adm[j]);
        carry = lab[j];
    }
    if (!d.forward_only) {
        carry = 0;
#pragma unroll
        for (int j = kWhole - 1; j >= 0; --j) {
            lab[j] |= carry & adm[j];
            carry = lab[j];
        }
    }
#pragma unroll
    for (int j = 0; j < kWhole; ++j) lab[j] &= ~cur[j];  // the new bits
    // the voxels that gained bits in any word, each marked once, by lane
    // jj & 7 of the particle's group: four per lane at most, in one batch
    // after both halves
    uint32_t marks[4] = {kNoVoxel, kNoVoxel, kNoVoxel, kNoVoxel};
#pragma unroll
    for (int h = 0; h < kWhole; h += 16) {
        uint32_t bb[16];
        uint64_t vv[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int j = h + jj;
            bb[jj] = kNoVoxel;
            if (lab[j]) atomicOr(&d.pplanes[((uint64_t)j * d.P + p) * 8 + k], lab[j]);
            const bool gnew = ((__ballot(lab[j] != 0) >> (8 * grp)) & 0xFFull) != 0;
            if (gnew) bb[jj] = bin[j];
        }
        uint32_t rv[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            vv[jj] = ~0ull;
            rv[jj] = 0u;
            if (bb[jj] != kNoVoxel) {
                int x, y, z, tt;
                bit_to_xyzt(d.g, bb[jj], x, y, z, tt);
                vv[jj] = vindex(d, x, y, z, tt);
                if (lab[h + jj]) rv[jj] = d.vrank[vv[jj]];
            }
        }
        uint32_t got[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            got[jj] = 0;
            if (vv[jj] != ~0ull && lab[h + jj]) {
                const uint32_t pw = lab[h + jj] & rank_word(s_ftab, rv[jj], k);
                if (pw) got[jj] = ~atomicOr(&d.fplanes[vv[jj] * 8 + k], pw) & pw;
            }
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const uint32_t gg = (uint32_t)(__ballot(got[jj] != 0) >> (8 * grp)) & 0xFFu;
            if (gg && (jj & 7) == k) marks[(h >> 3) + (jj >> 3)] = bb[jj];
        }
    }
    bmark_voxels_n<4>(d, marks, npar);
}

__global__ __launch_bounds__(256) void kb_close(DevB d, int par) {
    __shared__ uint32_t s_ptab[kLdsTab];
    __shared__ uint32_t s_ftab[kLdsTab];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (!d.counters[BC_RACT]) return;
    // the swept list is empty again (the close runs in every round, with or
    // without particles; the next list of this parity is built after the
    // round after this one)
    if (blockIdx.x == 0 && threadIdx.x < kBSubs) d.wcnt[((uint32_t)par * kBSubs + threadIdx.x) * kBCntStride] = 0u;
    for (uint32_t i = tid; i < d.NTB; i += stride) d.chg[par * d.NTB + i] = 0;
    const uint32_t nd = d.counters[BC_NDIRTYP];
    if (tid == 0 && nd) atomicAdd(&d.stat64[S_PART_VISITS], (unsigned long long)nd);
    const uint32_t per_block = (blockDim.x >> 6) * 8;
    if ((uint64_t)blockIdx.x * per_block >= nd) return;  // block-uniform
    stage_tables(d, 1, s_ptab);
    stage_tables(d, 0, s_ftab);
    __syncthreads();
    const int lane = lane_id(), k = lane & 7, grp = lane >> 3;
    const int npar = par ^ 1;
    const int ndir = d.forward_only ? 1 : 2;
    const int nch = (d.Tp + kChunk - 1) / kChunk;
    const uint32_t wave = tid >> 6, nwaves = stride >> 6;
    for (uint32_t base = wave * 8; base < nd; base += nwaves * 8) {  // wave-uniform
        const uint32_t i = base + grp;
        const bool valid = i < nd;
        const uint32_t p = valid ? d.dlist[i] : 0u;
        if (valid && k == 0) atomicAnd(&d.pdirty[p >> 5], ~(1u << (p & 31)));
        if (d.Tp <= kWhole) {
            close_whole(d, p, valid, k, grp, npar, s_ptab, s_ftab);
            continue;
        }
        for (int dir = 0; dir < ndir; ++dir) {
            uint32_t carry = 0;
            for (int ci = 0; ci < nch; ++ci) {
                const int c0 = (dir == 0 ? ci : nch - 1 - ci) * kChunk;
                const int cn = d.Tp - c0 < kChunk ? d.Tp - c0 : kChunk;
                uint32_t cur[kChunk], rk[kChunk], bb[kChunk];
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    cur[j] = 0;
                    rk[j] = 0;
                    bb[j] = kNoVoxel;
                    if (valid && j < cn) {
                        const uint64_t e = (uint64_t)p * d.Tpad + c0 + j;
                        cur[j] = d.pplanes[((uint64_t)(c0 + j) * d.P + p) * 8 + k];
                        rk[j] = d.prank[e];
                        bb[j] = d.bins[e];
                    }
                }
                uint32_t nw[kChunk];
#pragma unroll
                for (int jj = 0; jj < kChunk; ++jj) {
                    const int j = dir == 0 ? jj : kChunk - 1 - jj;
                    nw[j] = 0;
                    if (j < cn) {
                        const uint32_t l = cur[j] | (carry & rank_word(s_ptab, rk[j], k));
                        nw[j] = l & ~cur[j];
                        carry = l;
                    }
                }
                // new bits: the labels, then the pushed voxels' ranks, then
                // their label atomics, each for the whole chunk at once
                uint64_t vv[kChunk];
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    if (nw[j]) atomicOr(&d.pplanes[((uint64_t)(c0 + j) * d.P + p) * 8 + k], nw[j]);
                    const bool gnew = ((__ballot(nw[j] != 0) >> (8 * grp)) & 0xFFull) != 0;
                    vv[j] = ~0ull;
                    if (gnew && bb[j] != kNoVoxel) {
                        int x, y, z, tt;
                        bit_to_xyzt(d.g, bb[j], x, y, z, tt);
                        vv[j] = vindex(d, x, y, z, tt);
                    }
                }
                uint32_t rv[kChunk];
#pragma unroll
                for (int j = 0; j < kChunk; ++j) rv[j] = vv[j] != ~0ull && nw[j] ? d.vrank[vv[j]] : 0u;
                uint32_t got[kChunk];
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    got[j] = 0;
                    if (vv[j] != ~0ull && nw[j]) {
                        const uint32_t pw = nw[j] & rank_word(s_ftab, rv[j], k);
                        if (pw) got[j] = ~atomicOr(&d.fplanes[vv[j] * 8 + k], pw) & pw;
                    }
                }
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    const uint32_t gg = (uint32_t)(__ballot(got[j] != 0) >> (8 * grp)) & 0xFFu;
                    if (got[j] && k == __builtin_ctz(gg)) {
                        int x, y, z, tt;
                        bit_to_xyzt(d.g, bb[j], x, y, z, tt);
                        bmark_voxel(d, x, y, z, tt, npar);
                    }
                }
            }
        }
    }
}

// The work list of the round of parity `par` from the tiles flagged for it
// (the flags cleared for that parity's next use): a flagged tile joins if it
// holds a node admissible for some query.  Appends go to sub-list (tile mod
// kBSubs): 64 counters on separate lines.  force: also after a round without
// work (the list after seeding).
__global__ __launch_bounds__(256) void kb_compact(DevB d, int par, int force) {
    if (!force && !d.counters[BC_RACT]) return;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < d.NTB; i += stride) {
        uint32_t* f = &d.dirty[(size_t)par * d.NTB + i];
        if (*f) {
            *f = 0u;
            if (d.active[i]) {
                const uint32_t j = (uint32_t)par * kBSubs + (i & (kBSubs - 1));
                const uint32_t k = atomicAdd(&d.wcnt[j * kBCntStride], 1u);
                d.work[(size_t)j * d.WCAPB + k] = i;
            }
        }
    }
}

// Total length of the work list of parity par, for the host.
__global__ void kb_work_total(DevB d, int par) {
    uint32_t x = d.wcnt[((uint32_t)par * kBSubs + threadIdx.x) * kBCntStride];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (threadIdx.x == 0) d.counters[BC_NWORK0 + par] = x;
}

__global__ void kb_reset(DevB d) {
    const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = tid; i < 2ull * d.NTB; i += stride) d.dirty[i] = 0;
    for (uint64_t i = tid; i < (2ull * d.NTB + 3) / 4; i += stride)
        reinterpret_cast<uint32_t*>(d.chg)[i] = 0;
    for (uint64_t i = tid; i < ((uint64_t)d.NTB + 3) / 4; i += stride)
        reinterpret_cast<uint32_t*>(d.active)[i] = 0;
    for (uint64_t i = tid; i < (uint64_t)(d.P + 31) / 32; i += stride) d.pdirty[i] = 0;
    if (tid < BC_NCOUNTERS) d.counters[tid] = 0;
    if (tid < 2 * kBSubs) d.wcnt[tid * kBCntStride] = 0;
    if (tid < S_NSTAT) d.stat64[tid] = 0;
}

__global__ void kb_count(DevB d) {
    const uint64_t nf = (uint64_t)d.X * d.Y * d.Z * d.T * 8;
    const uint64_t np = (uint64_t)d.Tp * d.P * 8;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long cf = 0, cp = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nf; i += stride)
        cf += __popc(d.fplanes[i]);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < np; i += stride)
        cp += __popc(d.pplanes[i]);
    for (int o = 32; o > 0; o >>= 1) {
        cf += __shfl_xor(cf, o);
        cp += __shfl_xor(cp, o);
    }
    if (lane_id() == 0) {
        if (cf) atomicAdd(&d.stat64[S_MEMBERS_F], cf);
        if (cp) atomicAdd(&d.stat64[S_MEMBERS_P], cp);
    }
}

inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap) {
    uint64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

void launch_b_prepare(const DevB& d, const int32_t* seeds, int64_t S, hipStream_t s) {
    const uint64_t V = (uint64_t)d.X * d.Y * d.Z * d.T;
    hipLaunchKernelGGL(kb_reset, dim3(grid_for(2ull * d.NTB + d.P / 32 + 1, 256, 2048)), dim3(256),
                       0, s, d);
    hipLaunchKernelGGL(kb_admit_field, dim3(grid_for(V, 256, 4096)), dim3(256), 0, s, d);
    if (d.P > 0)
        hipLaunchKernelGGL(kb_admit_particles,
                           dim3(grid_for((uint64_t)d.P * d.Tpad, 256, 8192)), dim3(256), 0, s, d);
    if (S > 0)
        hipLaunchKernelGGL(kb_seeds, dim3(grid_for(S, 256, 1u << 20)), dim3(256), 0, s, d, seeds, S);
    hipLaunchKernelGGL(kb_compact, dim3(grid_for(d.NTB, 256, 1024)), dim3(256), 0, s, d, 0, 1);
}

void launch_b_round(const DevB& d, uint32_t round, hipStream_t s) {
    const int par = round & 1;
    if (d.lx == 2 && d.ly == 2 && d.lz == 2)
        hipLaunchKernelGGL(kb_sweep<true>, dim3(grid_for(d.NTB, 1, 2048)), dim3(512), 0, s, d, par);
    else
        hipLaunchKernelGGL(kb_sweep<false>, dim3(grid_for(d.NTB, 1, 2048)), dim3(512), 0, s, d, par);
    if (d.P > 0) {
        hipLaunchKernelGGL(kb_pull, dim3(grid_for((uint64_t)d.P * d.Tpad, 256, 2048)), dim3(256), 0,
                           s, d, par);
        const uint64_t nclose = (uint64_t)d.NTB > (uint64_t)d.P ? (uint64_t)d.NTB : (uint64_t)d.P;
        hipLaunchKernelGGL(kb_close, dim3(grid_for(nclose, 256, 2048)), dim3(256), 0, s, d, par);
    } else {
        hipLaunchKernelGGL(kb_close, dim3(grid_for(d.NTB, 256, 2048)), dim3(256), 0, s, d, par);
    }
    hipLaunchKernelGGL(kb_compact, dim3(grid_for(d.NTB, 256, 1024)), dim3(256), 0, s, d, par ^ 1, 0);
}

void launch_b_work_total(const DevB& d, int par, hipStream_t s) {
    hipLaunchKernelGGL(kb_work_total, dim3(1), dim3(64), 0, s, d, par);
}

void launch_b_count(const DevB& d, hipStream_t s) {
    const uint64_t V = (uint64_t)d.X * d.Y * d.Z * d.T;
    hipLaunchKernelGGL(kb_count, dim3(grid_for(V * 8, 256, 8192)), dim3(256), 0, s, d);
}

}  // namespace mf4d
