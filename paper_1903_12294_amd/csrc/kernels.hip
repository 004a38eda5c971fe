// HIP kernels of the coupled point + field region grower, for gfx950 (wave64).
//
// Field nodes are kept as bit-packed tiles (see Geom in mf4d_internal.h); the
// particle part as one bit per particle-step in 64-bit words per particle.
// Every label bit only goes 0 -> 1, so the order in which waves apply their
// updates cannot change the fixed point they reach.
#include "mf4d_internal.h"

namespace mf4d {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Index in a wave-wide append of the lanes with pred set: one atomicAdd per wave.
// Every lane of the wave must call it.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* counter) {
    const uint64_t m = __ballot(pred);
    if (m == 0) return 0;
    const int lane = lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

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

// A voxel bit set from outside a tile sweep (seed or particle push): its own
// tile must be swept, and so must every tile whose face it touches, because
// the owning tile's sweep only reports bits that are new to that sweep.
__device__ void mark_voxel(const Geom& g, uint32_t b, const uint8_t* active, uint8_t* dirty) {
    const uint32_t word = b >> 5;
    const int xb = b & 31;
    const uint32_t tile = word >> (6 + g.logBT);
    const uint32_t wi = word & (g.WPT - 1);
    const int yl = wi & 7, zl = (wi >> 3) & 7, tl = wi >> 6;
    dirty[tile] = 1;
    int tx, ty, tz, tt;
    tile_coords(g, tile, tx, ty, tz, tt);
    const uint32_t sy = g.NXt, sz = g.NXt * g.NYt, st = sz * g.NZt;
    uint32_t nb[4];
    int k = 0;
    if (xb == 0 && tx > 0) nb[k++] = tile - 1;
    if (xb == 31 && tx + 1 < g.NXt) nb[k++] = tile + 1;
    if (yl == 0 && ty > 0) nb[k++] = tile - sy;
    if (yl == 7 && ty + 1 < g.NYt) nb[k++] = tile + sy;
    for (int i = 0; i < k; ++i)
        if (active[nb[i]]) dirty[nb[i]] = 1;
    k = 0;
    if (zl == 0 && tz > 0) nb[k++] = tile - sz;
    if (zl == 7 && tz + 1 < g.NZt) nb[k++] = tile + sz;
    if (tl == 0 && tt > 0) nb[k++] = tile - st;
    if (tl == g.BT - 1 && tt + 1 < g.NTt) nb[k++] = tile + st;
    for (int i = 0; i < k; ++i)
        if (active[nb[i]]) dirty[nb[i]] = 1;
}

__device__ __forceinline__ bool test_bit(const uint32_t* a, uint32_t b) {
    return (a[b >> 5] >> (b & 31)) & 1u;
}

// ---------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Load: bin every particle-step into the voxel covering it and transpose the
// values to particle-major rows.  Block = 64 particles; LDS tile [64][65].
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
                    b = bit_index(g, (int)cx, (int)cy, (int)cz, t);
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

// Admissibility of every voxel-step, bit-packed into tiles.  Block = 256
// threads for the 64 rows (z_l, y_l) of one (t, tz, ty); x in passes of 256.
// Each lane tests 4 consecutive x; 8 lanes OR their nibbles into one word.
__global__ __launch_bounds__(256) void k_admit_field(Geom g, const float* __restrict__ f, float lo,
                                                     float hi, uint32_t* __restrict__ A,
                                                     uint8_t* __restrict__ active) {
    __shared__ uint32_t sw[8 * 64];
    const int ty = blockIdx.x, tz = blockIdx.y, t = blockIdx.z;
    const int tt = t >> g.logBT, tl = t & (g.BT - 1);
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const bool vec = (g.X & 3) == 0;
    for (int tx0 = 0; tx0 < g.NXt; tx0 += 8) {
        const int ntx = min(8, g.NXt - tx0);
        const int x = tx0 * 32 + 4 * lane;
        float4 v[16];
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int row = wave * 16 + rr;
            const int y = ty * 8 + (row & 7), z = tz * 8 + (row >> 3);
            v[rr] = make_float4(__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""),
                                __builtin_nanf(""));
            if (y < g.Y && z < g.Z) {
                const float* rp = f + ((size_t)(t * g.Z + z) * g.Y + y) * g.X;
                if (vec) {
                    if (x < g.X) v[rr] = *reinterpret_cast<const float4*>(rp + x);
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
            uint32_t nib = (uint32_t)in_band(v[rr].x, lo, hi) |
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
            A[(size_t)tile * g.WPT + tl * 64 + row] = w;
            if (__ballot(w != 0) != 0 && lane == 0) active[tile] = 1;
        }
        __syncthreads();
    }
}

__global__ void k_count_active(Geom g, const uint8_t* __restrict__ active,
                               unsigned long long* stat) {
    uint32_t c = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < g.NT; i += gridDim.x * blockDim.x)
        c += active[i];
    const uint64_t m = __ballot(c != 0);
    // reduce counts across the wave
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane_id() == 0 && m) atomicAdd(stat, (unsigned long long)c);
}

// Admissibility of every particle-step: one ballot per 64 flat steps gives the
// step bits of one word (or of 64 / Tpad particles).  Admissible steps that lie
// in a voxel are appended to the coupled list (flat index, voxel bit).
__global__ __launch_bounds__(256) void k_admit_particles(PGeom pg, const float* __restrict__ at,
                                                         const uint32_t* __restrict__ bins,
                                                         float lo, float hi,
                                                         unsigned long long* __restrict__ Ap,
                                                         uint2* __restrict__ pend,
                                                         uint32_t* __restrict__ npend) {
    const uint64_t n = (uint64_t)pg.P * pg.Tpad;
    const int lane = lane_id();
    const uint64_t wave0 = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t base = wave0 * 256; base < n; base += nwaves * 256) {
        float a[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t e = base + k * 64 + lane;
            a[k] = e < n ? at[e] : __builtin_nanf("");
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t e0 = base + k * 64;
            const uint64_t e = e0 + lane;
            const bool adm = in_band(a[k], lo, hi);
            const uint64_t m = __ballot(adm);
            if (e0 < n) {
                if (pg.Tpad >= 64) {
                    if (lane == 0) Ap[e0 >> 6] = m;
                } else {
                    const int per = 64 >> pg.logTpad;
                    if (lane < per) {
                        const uint64_t p = (e0 >> pg.logTpad) + lane;
                        if (p < (uint64_t)pg.P)
                            Ap[p] = (m >> (lane * pg.Tpad)) & ((1ull << pg.Tpad) - 1ull);
                    }
                }
            }
            const uint32_t b = adm ? bins[e] : kNoVoxel;
            const bool c = adm && b != kNoVoxel;
            const uint32_t idx = wave_append(c, npend);
            if (c) pend[idx] = make_uint2((uint32_t)e, b);
        }
    }
}

__global__ void k_seeds(Geom g, const int32_t* __restrict__ seeds, int64_t S,
                        const uint32_t* __restrict__ A, uint32_t* L,
                        const uint8_t* __restrict__ active, uint8_t* dirty, uint32_t* dropped) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= S) return;
    const int32_t* s = seeds + 4 * i;
    const uint32_t b = bit_index(g, s[0], s[1], s[2], s[3]);
    if (test_bit(A, b)) {
        const uint32_t bit = 1u << (b & 31);
        const uint32_t old = atomicOr(&L[b >> 5], bit);
        if (!(old & bit)) mark_voxel(g, b, active, dirty);
    } else {
        atomicAdd(dropped, 1u);
    }
}

// Dirty tile flags -> compact work list (ballot prefix, one atomic per wave).
__global__ void k_compact_tiles(uint32_t NT, uint8_t* __restrict__ dirty, uint32_t* __restrict__ work,
                                uint32_t* nwork) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < NT; base += stride) {
        const uint32_t i = base + threadIdx.x;
        bool d = false;
        if (i < NT) {
            d = dirty[i] != 0;
            if (d) dirty[i] = 0;
        }
        const uint32_t idx = wave_append(d, nwork);
        if (d) work[idx] = i;
    }
}

// Put a work list back as dirty flags (a round cap stopped before sweeping it).
__global__ void k_mark_work(const uint32_t* __restrict__ work, const uint32_t* __restrict__ nwork_p,
                            uint8_t* dirty) {
    const uint32_t n = *nwork_p;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dirty[work[i]] = 1;
}

// One wavefront sweeps one tile to a local fixed point.  Lane = (z_l, y_l);
// each lane holds the BT words of its (y, z) column over the tile's timesteps
// in registers.  Per iteration: one Jacobi step in y and z (lane shuffles),
// complete fills along x inside each word, and complete forward / backward
// passes along t.  Neighbour-tile words enter as fixed halos; when a face of
// this tile gains bits, the tile across that face is marked for the next round.
template <int BT>
__global__ __launch_bounds__(256) void k_sweep(Geom g, const uint32_t* __restrict__ A, uint32_t* L,
                                               const uint8_t* __restrict__ active,
                                               const uint32_t* __restrict__ work,
                                               const uint32_t* __restrict__ nwork_p,
                                               uint8_t* dirty, unsigned long long* visits) {
    const int lane = lane_id();
    const int yl = lane & 7, zl = lane >> 3;
    const uint32_t nwork = *nwork_p;
    const uint32_t wave0 = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t sy = g.NXt, sz = g.NXt * g.NYt, st = sz * g.NZt;
    uint32_t myvisits = 0;
    for (uint32_t wi = wave0; wi < nwork; wi += nwaves) {
        const uint32_t tile = work[wi];
        int tx, ty, tz, tt;
        tile_coords(g, tile, tx, ty, tz, tt);
        const uint32_t* Ab = A + (size_t)tile * (64 * BT);
        uint32_t* Lb = L + (size_t)tile * (64 * BT);
        uint32_t a[BT], l[BT], l0[BT], xin[BT], yh[BT], zh[BT];
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            a[t] = Ab[t * 64 + lane];
            l[t] = Lb[t * 64 + lane];
        }
        const uint32_t* Lxm = tx > 0 ? Lb - 64 * BT : nullptr;
        const uint32_t* Lxp = tx + 1 < g.NXt ? Lb + 64 * BT : nullptr;
        const uint32_t* Ly = nullptr;
        int yoff = 0;
        if (yl == 0 && ty > 0) { Ly = Lb - (size_t)sy * 64 * BT; yoff = 7; }
        if (yl == 7 && ty + 1 < g.NYt) { Ly = Lb + (size_t)sy * 64 * BT; yoff = -7; }
        const uint32_t* Lz = nullptr;
        int zoff = 0;
        if (zl == 0 && tz > 0) { Lz = Lb - (size_t)sz * 64 * BT; zoff = 56; }
        if (zl == 7 && tz + 1 < g.NZt) { Lz = Lb + (size_t)sz * 64 * BT; zoff = -56; }
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            xin[t] = (Lxm ? (Lxm[t * 64 + lane] >> 31) : 0u) | (Lxp ? (Lxp[t * 64 + lane] << 31) : 0u);
            yh[t] = Ly ? Ly[t * 64 + lane + yoff] : 0u;
            zh[t] = Lz ? Lz[t * 64 + lane + zoff] : 0u;
            l0[t] = l[t];
        }
        const uint32_t tm = tt > 0 ? (Lb - (size_t)st * 64 * BT)[(BT - 1) * 64 + lane] : 0u;
        const uint32_t tp = tt + 1 < g.NTt ? (Lb + (size_t)st * 64 * BT)[lane] : 0u;
        while (true) {
            uint32_t s[BT];
#pragma unroll
            for (int t = 0; t < BT; ++t) {
                const uint32_t v = l[t];
                const uint32_t ym = __shfl_up(v, 1), yp = __shfl_down(v, 1);
                const uint32_t zm = __shfl_up(v, 8), zp = __shfl_down(v, 8);
                uint32_t nb = v | (v << 1) | (v >> 1) | xin[t] | yh[t] | zh[t];
                nb |= (yl > 0 ? ym : 0u) | (yl < 7 ? yp : 0u) | (zl > 0 ? zm : 0u) |
                      (zl < 7 ? zp : 0u);
                s[t] = fill_runs32(nb & a[t], a[t]);
            }
            s[0] |= fill_runs32(tm & a[0], a[0]);
#pragma unroll
            for (int t = 1; t < BT; ++t) s[t] |= fill_runs32(s[t - 1] & a[t], a[t]);
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
        uint32_t any = 0, fx0 = 0, fx1 = 0;
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            const uint32_t nw = l[t] & ~l0[t];
            if (nw) atomicOr(&Lb[t * 64 + lane], nw);
            any |= nw;
            fx0 |= nw & 1u;
            fx1 |= nw >> 31;
        }
        const uint32_t nt0 = l[0] & ~l0[0], nt1 = l[BT - 1] & ~l0[BT - 1];
        const uint64_t b_any = __ballot(any != 0);
        if (b_any) {
            const bool fxm = __ballot(fx0 != 0) != 0, fxp = __ballot(fx1 != 0) != 0;
            const bool fym = __ballot(yl == 0 && any) != 0, fyp = __ballot(yl == 7 && any) != 0;
            const bool fzm = __ballot(zl == 0 && any) != 0, fzp = __ballot(zl == 7 && any) != 0;
            const bool ftm = __ballot(nt0 != 0) != 0, ftp = __ballot(nt1 != 0) != 0;
            if (lane == 0) {
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
                for (int i = 0; i < k; ++i)
                    if (active[nb[i]]) dirty[nb[i]] = 1;
            }
        }
        ++myvisits;
    }
    if (lane == 0 && myvisits) atomicAdd(visits, (unsigned long long)myvisits);
}

// Pull: a pending coupled particle-step joins when the voxel holding it is a
// member.  Steps that joined (now or earlier) leave the pending list; a
// particle that gained a step goes on the dirty-particle list once.
__global__ __launch_bounds__(256) void k_pull(PGeom pg, const uint2* __restrict__ pin,
                                              const uint32_t* __restrict__ nin_p,
                                              uint2* __restrict__ pout, uint32_t* nout,
                                              const uint32_t* __restrict__ Lf,
                                              unsigned long long* Lp, uint32_t* pdirty,
                                              uint32_t* dlist, uint32_t* ndlist) {
    const uint32_t nin = *nin_p;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < nin; base += stride) {
        const uint32_t i = base + threadIdx.x;
        bool keep = false, first = false;
        uint2 ent = make_uint2(0, 0);
        uint32_t p = 0;
        if (i < nin) {
            ent = pin[i];
            const uint32_t e = ent.x;
            uint32_t t;
            if (pg.logTpad >= 0) {
                p = e >> pg.logTpad;
                t = e & (pg.Tpad - 1);
            } else {
                p = e / (uint32_t)pg.Tpad;
                t = e - p * (uint32_t)pg.Tpad;
            }
            const uint32_t wi = p * (uint32_t)pg.W + (t >> 6);
            const unsigned long long bit = 1ull << (t & 63);
            if (!(Lp[wi] & bit)) {
                if (test_bit(Lf, ent.y)) {
                    atomicOr(&Lp[wi], bit);
                    const uint32_t pb = 1u << (p & 31);
                    first = !(atomicOr(&pdirty[p >> 5], pb) & pb);
                } else {
                    keep = true;
                }
            }
        }
        const uint32_t k = wave_append(keep, nout);
        if (keep) pout[k] = ent;
        const uint32_t d = wave_append(first, ndlist);
        if (first) dlist[d] = p;
    }
}

// Close and push: a dirty particle's member steps spread over each run of
// admissible steps that holds them (its trajectory), and every step that
// joins pushes its voxel in when that voxel is admissible.
__global__ __launch_bounds__(256) void k_close_push(Geom g, PGeom pg, const uint32_t* __restrict__ dlist,
                                                    const uint32_t* __restrict__ nd_p,
                                                    const unsigned long long* __restrict__ Ap,
                                                    unsigned long long* Lp, uint32_t* pdirty,
                                                    const uint32_t* __restrict__ bins,
                                                    const uint32_t* __restrict__ Af, uint32_t* Lf,
                                                    const uint8_t* __restrict__ active,
                                                    uint8_t* dirty, unsigned long long* visits) {
    const uint32_t nd = *nd_p;
    if (blockIdx.x == 0 && threadIdx.x == 0 && nd) atomicAdd(visits, (unsigned long long)nd);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x) {
        const uint32_t p = dlist[i];
        atomicAnd(&pdirty[p >> 5], ~(1u << (p & 31)));
        const int W = pg.W;
        unsigned long long* lw = Lp + (size_t)p * W;
        const unsigned long long* aw = Ap + (size_t)p * W;
        // forward pass (carry over word boundaries upward), then backward
        unsigned long long carry = 0;
        for (int w = 0; w < W; ++w) {
            const unsigned long long a = aw[w], l0 = lw[w];
            unsigned long long l = l0 | (carry & a & 1ull);
            l = fill_runs64(l, a);
            carry = l >> 63;
            const unsigned long long nw = l & ~l0;
            if (nw) {
                atomicOr(&lw[w], nw);
                unsigned long long m = nw;
                while (m) {
                    const int t = __builtin_ctzll(m);
                    m &= m - 1;
                    const uint32_t b = bins[(size_t)p * pg.Tpad + w * 64 + t];
                    if (b != kNoVoxel && test_bit(Af, b)) {
                        const uint32_t bit = 1u << (b & 31);
                        if (!(atomicOr(&Lf[b >> 5], bit) & bit)) mark_voxel(g, b, active, dirty);
                    }
                }
            }
        }
        carry = 0;
        for (int w = W - 1; w >= 0; --w) {
            const unsigned long long a = aw[w], l0 = lw[w];
            unsigned long long l = l0 | ((carry << 63) & a);
            l = fill_runs64(l, a);
            carry = l & 1ull;
            const unsigned long long nw = l & ~l0;
            if (nw) {
                atomicOr(&lw[w], nw);
                unsigned long long m = nw;
                while (m) {
                    const int t = __builtin_ctzll(m);
                    m &= m - 1;
                    const uint32_t b = bins[(size_t)p * pg.Tpad + w * 64 + t];
                    if (b != kNoVoxel && test_bit(Af, b)) {
                        const uint32_t bit = 1u << (b & 31);
                        if (!(atomicOr(&Lf[b >> 5], bit) & bit)) mark_voxel(g, b, active, dirty);
                    }
                }
            }
        }
    }
}

// Field labels -> canonical bit words ((t*Z + z)*Y + y)*X + x, with a member
// count.  Fast path when X is a multiple of 32 (a canonical word is one tile
// word); otherwise bit by bit.
__global__ __launch_bounds__(256) void k_read_field(Geom g, const uint32_t* __restrict__ L,
                                                    uint32_t* __restrict__ out,
                                                    unsigned long long* members) {
    const uint64_t V = (uint64_t)g.X * g.Y * g.Z * g.T;
    const uint64_t nw = (V + 31) >> 5;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t cnt = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nw; i += stride) {
        uint32_t w = 0;
        if ((g.X & 31) == 0) {
            const uint32_t wpr = g.X >> 5;
            const uint32_t row = (uint32_t)(i / wpr);
            const int x0 = (int)(i - (uint64_t)row * wpr) * 32;
            const int y = row % g.Y;
            const uint32_t r2 = row / g.Y;
            const int z = r2 % g.Z, t = r2 / g.Z;
            w = L[bit_index(g, x0, y, z, t) >> 5];
        } else {
            for (int k = 0; k < 32; ++k) {
                const uint64_t bi = i * 32 + k;
                if (bi >= V) break;
                const uint32_t x = (uint32_t)(bi % g.X);
                const uint64_t r = bi / g.X;
                const int y = r % g.Y;
                const uint64_t r2 = r / g.Y;
                const int z = r2 % g.Z, t = (int)(r2 / g.Z);
                if (test_bit(L, bit_index(g, (int)x, y, z, t))) w |= 1u << k;
            }
        }
        out[i] = w;
        cnt += __popc(w);
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane_id() == 0 && cnt) atomicAdd(members, (unsigned long long)cnt);
}

// Particle labels -> uint8 [T][P].  A thread owns 4 consecutive particles and
// writes their 4 bytes per timestep as one 32-bit store when aligned.
__global__ __launch_bounds__(256) void k_read_particles(PGeom pg, const unsigned long long* __restrict__ Lp,
                                                        uint8_t* __restrict__ out,
                                                        unsigned long long* members) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t p0 = q * 4;
    uint32_t cnt = 0;
    if (p0 < pg.P) {
        const int np = (int)min((int64_t)4, pg.P - p0);
        const bool vec = np == 4 && (pg.P & 3) == 0;
        for (int w = 0; w < pg.W; ++w) {
            unsigned long long lw[4] = {0, 0, 0, 0};
            for (int k = 0; k < np; ++k) {
                lw[k] = Lp[(size_t)(p0 + k) * pg.W + w];
                cnt += __popcll(lw[k]);
            }
            const int tend = min(64, pg.T - w * 64);
            for (int tl = 0; tl < tend; ++tl) {
                const int64_t t = w * 64 + tl;
                uint8_t* o = out + t * pg.P + p0;
                if (vec) {
                    const uint32_t v = (uint32_t)((lw[0] >> tl) & 1) | ((uint32_t)((lw[1] >> tl) & 1) << 8) |
                                       ((uint32_t)((lw[2] >> tl) & 1) << 16) |
                                       ((uint32_t)((lw[3] >> tl) & 1) << 24);
                    *reinterpret_cast<uint32_t*>(o) = v;
                } else {
                    for (int k = 0; k < np; ++k) o[k] = (uint8_t)((lw[k] >> tl) & 1);
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane_id() == 0 && cnt) atomicAdd(members, (unsigned long long)cnt);
}

inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap) {
    uint64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
}

void launch_bin_particles(const Geom& g, const PGeom& pg, const float* xyz, const float* attr,
                          uint32_t* bins, float* attr_t, hipStream_t s) {
    if (pg.P == 0) return;
    const unsigned nb = (unsigned)((pg.P + 63) / 64);
    hipLaunchKernelGGL(k_bin_particles, dim3(nb), dim3(256), 0, s, g, pg, xyz, attr, bins, attr_t);
}

void launch_admit_field(const Geom& g, const float* field, float lo, float hi, uint32_t* A,
                        uint8_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_admit_field, dim3(g.NYt, g.NZt, g.T), dim3(256), 0, s, g, field, lo, hi,
                       A, active);
}

void launch_count_active(const Geom& g, const uint8_t* active, unsigned long long* stat,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_count_active, dim3(grid_for(g.NT, 256, 1024)), dim3(256), 0, s, g, active,
                       stat);
}

void launch_admit_particles(const PGeom& pg, const float* attr_t, const uint32_t* bins, float lo,
                            float hi, unsigned long long* Ap, uint2* pend, uint32_t* npend,
                            hipStream_t s) {
    const uint64_t n = (uint64_t)pg.P * pg.Tpad;
    if (n == 0) return;
    hipLaunchKernelGGL(k_admit_particles, dim3(grid_for(n / 4, 256, 16384)), dim3(256), 0, s, pg,
                       attr_t, bins, lo, hi, Ap, pend, npend);
}

void launch_seeds(const Geom& g, const int32_t* seeds, int64_t S, const uint32_t* A, uint32_t* L,
                  const uint8_t* active, uint8_t* dirty, uint32_t* dropped, hipStream_t s) {
    if (S == 0) return;
    hipLaunchKernelGGL(k_seeds, dim3(grid_for(S, 256, 1u << 20)), dim3(256), 0, s, g, seeds, S, A,
                       L, active, dirty, dropped);
}

void launch_compact_tiles(const Geom& g, uint8_t* dirty, uint32_t* work, uint32_t* nwork,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_compact_tiles, dim3(grid_for(g.NT, 256, 2048)), dim3(256), 0, s, g.NT,
                       dirty, work, nwork);
}

void launch_mark_work(const uint32_t* work, const uint32_t* nwork, uint32_t nwork_host,
                      uint8_t* dirty, hipStream_t s) {
    if (nwork_host == 0) return;
    hipLaunchKernelGGL(k_mark_work, dim3(grid_for(nwork_host, 256, 4096)), dim3(256), 0, s, work,
                       nwork, dirty);
}

void launch_sweep(const Geom& g, const uint32_t* A, uint32_t* L, const uint8_t* active,
                  const uint32_t* work, const uint32_t* nwork, uint32_t nwork_host,
                  uint8_t* dirty, unsigned long long* visits, hipStream_t s) {
    if (nwork_host == 0) return;
    const unsigned blocks = grid_for((uint64_t)nwork_host * 64, 256, 8192);
    switch (g.BT) {
        case 4:
            hipLaunchKernelGGL(k_sweep<4>, dim3(blocks), dim3(256), 0, s, g, A, L, active, work,
                               nwork, dirty, visits);
            break;
        case 8:
            hipLaunchKernelGGL(k_sweep<8>, dim3(blocks), dim3(256), 0, s, g, A, L, active, work,
                               nwork, dirty, visits);
            break;
        default:
            hipLaunchKernelGGL(k_sweep<16>, dim3(blocks), dim3(256), 0, s, g, A, L, active, work,
                               nwork, dirty, visits);
            break;
    }
}

void launch_pull(const PGeom& pg, const uint2* pin, const uint32_t* nin, uint32_t nin_host,
                 uint2* pout, uint32_t* nout, const uint32_t* Lf, unsigned long long* Lp,
                 uint32_t* pdirty, uint32_t* dlist, uint32_t* ndlist, hipStream_t s) {
    if (nin_host == 0) return;
    hipLaunchKernelGGL(k_pull, dim3(grid_for(nin_host, 256, 8192)), dim3(256), 0, s, pg, pin, nin,
                       pout, nout, Lf, Lp, pdirty, dlist, ndlist);
}

void launch_close_push(const Geom& g, const PGeom& pg, const uint32_t* dlist,
                       const uint32_t* ndlist, uint32_t ndlist_host,
                       const unsigned long long* Ap, unsigned long long* Lp, uint32_t* pdirty,
                       const uint32_t* bins, const uint32_t* Af, uint32_t* Lf,
                       const uint8_t* active, uint8_t* dirty, unsigned long long* visits,
                       hipStream_t s) {
    if (ndlist_host == 0) return;
    hipLaunchKernelGGL(k_close_push, dim3(grid_for(ndlist_host, 256, 2048)), dim3(256), 0, s, g,
                       pg, dlist, ndlist, Ap, Lp, pdirty, bins, Af, Lf, active, dirty, visits);
}

void launch_read_field(const Geom& g, const uint32_t* L, uint32_t* out,
                       unsigned long long* members, hipStream_t s) {
    const uint64_t V = (uint64_t)g.X * g.Y * g.Z * g.T;
    hipLaunchKernelGGL(k_read_field, dim3(grid_for((V + 31) / 32, 256, 16384)), dim3(256), 0, s, g,
                       L, out, members);
}

void launch_read_particles(const PGeom& pg, const unsigned long long* Lp, uint8_t* out,
                           unsigned long long* members, hipStream_t s) {
    if (pg.P == 0) return;
    hipLaunchKernelGGL(k_read_particles, dim3(grid_for((pg.P + 3) / 4, 256, 1u << 20)), dim3(256),
                       0, s, pg, Lp, out, members);
}

}  // namespace mf4d
