// 4D SLIC clustering of point and field samples (Section 3.2) on gfx950.
//
// One iteration is two fused passes (field samples, then point samples) and
// one small update.  A pass assigns each sample to the centre with the
// smallest distance among those whose window holds it (Section 3.2.2-3.2.3)
// and adds the sample's quantised coordinates and value to its centre's
// sums: first in a block-local LDS table keyed by centre (a block of 1024
// consecutive samples touches few centres), then with one 64-bit atomic per
// touched centre and sum.  Integer sums make the centres independent of the
// order of the additions, so they are bit-identical run to run.  The update
// turns the sums into means, compares them with the previous centres
// (convergence, Section 3.2.2) and clears the sums.
//
// Arithmetic that decides a label is IEEE fp32 with every operation rounded
// on its own (no fused multiply-add), in a fixed order:
//   S = sqrt(((dx*dx + dy*dy) + dz*dz) + (cf*dt)*(cf*dt)),  D = w_v*|v - v_c| + w_d*S.
#include "slic.h"

#include <math.h>

#include <algorithm>

namespace mf4d {
namespace {

constexpr double kQScale = 1048576.0;  // 2^20: quantisation of coordinates and values
constexpr double kQInv = 1.0 / 1048576.0;
constexpr float kMaxAbs = 2048.0f;     // |coordinate|, |value| below this keep the sums in int64
constexpr int kTab = 64;               // LDS table slots (centres one block touches)
constexpr int kBlock = 256;
constexpr int kPer = 4;                // samples per thread per pass

__device__ __forceinline__ int seed_cell(float pos, float C, int kd) {
    const float q = floorf(__fdiv_rn(pos, C));
    return (int)fminf(fmaxf(q, 0.0f), (float)(kd - 1));
}

__device__ __forceinline__ long long quantise(float v) {
    return __double2ll_rn((double)v * kQScale);
}

// dbl(s) = float64(s >> 32) * 2^32 + float64(s & 0xffffffff): the product is
// exact, so one rounding whether or not the two are fused.
__device__ __forceinline__ double to_double(long long s) {
    const double hi = (double)(int)(s >> 32);
    const double lo = (double)(unsigned)(s & 0xFFFFFFFFll);
    return hi * 4294967296.0 + lo;
}

// Order-preserving map of fp32 to uint32 (and back), for atomic min / max.
__device__ __forceinline__ uint32_t float_key(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Candidate search.  A centre's window holds a sample when |p_d - c_d| <=
// C_d on every axis (Section 3.2.2).  A centre may drift any distance from
// its seed cell, so no fixed neighbourhood of seed cells is assumed: after
// each update, per axis d, every slab i (the centres with cell index i on
// axis d) records the least and greatest coordinate of its centres, and every
// seed cell j the range reach[d][j] of slabs whose [least - C, greatest + C]
// meets cell j.  A sample of cell j then tests exactly those slabs.  Rounding
// of p - c is monotone in c, so a centre that passes the window test lies in
// a slab that passes the slab test: no candidate is lost.

__device__ __forceinline__ bool slab_holds(const DevS& s, int d, int i, float p) {
    const float lo = key_float(s.slab[(0 * 4 + d) * s.kmax + i]);
    const float hi = key_float(s.slab[(1 * 4 + d) * s.kmax + i]);
    return __fsub_rn(p, hi) <= s.C[d] && __fsub_rn(p, lo) >= -s.C[d];
}

// The slabs of axis d that can hold a centre within C of p (seed cell c), as
// bits i - base.  A reach range of more than s.mask_slabs (<= 32) slabs
// (centres drifted by many cells) sets `wide`: the caller then takes
// assign_wide.
__device__ __forceinline__ unsigned axis_mask(const DevS& s, int d, int c, float p, int& base, bool& wide) {
    const int lo = s.reach[(d * s.kmax + c) * 2], hi = s.reach[(d * s.kmax + c) * 2 + 1];
    base = lo;
    if (hi < lo) return 0u;
    if (hi - lo >= s.mask_slabs) {
        wide = true;
        return 0u;
    }
    unsigned m = 0;
    for (int i = lo; i <= hi; ++i)
        if (slab_holds(s, d, i, p)) m |= 1u << (i - lo);
    return m;
}

// Rate centre id for the sample if its window holds it; keep the smallest D,
// ties to the lowest id.
__device__ __forceinline__ void consider(const DevS& s, int id, float px, float py, float pz, float pt, float v,
                                         bool field, float wv, float& best_d, int& best) {
    const float4 c = reinterpret_cast<const float4*>(s.cen32)[2 * id];
    const float2 cv = reinterpret_cast<const float2*>(s.cen32)[4 * id + 2];
    const float dx = __fsub_rn(px, c.x), dy = __fsub_rn(py, c.y);
    const float dz = __fsub_rn(pz, c.z), dt = __fsub_rn(pt, c.w);
    if (!(fabsf(dx) <= s.C[0] && fabsf(dy) <= s.C[1] && fabsf(dz) <= s.C[2] && fabsf(dt) <= s.C[3])) return;
    const float vc = field ? cv.y : cv.x;
    const float A = __fmul_rn(wv, fabsf(__fsub_rn(v, vc)));
    // D = A + (w_d S) rounded is >= A: a value term above the best distance
    // cannot win (nor tie), so skip the rest
    if (A > best_d) return;
    const float ctd = __fmul_rn(s.cf, dt);
    const float sq = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz)),
                               __fmul_rn(ctd, ctd));
    const float D = __fadd_rn(A, __fmul_rn(s.wd, __fsqrt_rn(sq)));
    if (D < best_d || (D == best_d && id < best)) {
        best_d = D;
        best = id;
    }
}

// Centre with the smallest distance among the centres of the slabs in the
// masks (bit b of mx: slab bx0 + b on x, and so on); none: `prev`.
__device__ int assign_cands(const DevS& s, float px, float py, float pz, float pt, float v, bool field,
                            int prev, int bx0, int by0, int bz0, int bt0, unsigned mx, unsigned my,
                            unsigned mz, unsigned mt) {
    const float wv = field ? s.wf : s.wp;
    float best_d = INFINITY;
    int best = 0x7FFFFFFF;
    for (unsigned bt = mt; bt; bt &= bt - 1)
        for (unsigned bz = mz; bz; bz &= bz - 1)
            for (unsigned by = my; by; by &= by - 1)
                for (unsigned bx = mx; bx; bx &= bx - 1) {
                    const int ct = bt0 + __builtin_ctz(bt), cz = bz0 + __builtin_ctz(bz);
                    const int cy = by0 + __builtin_ctz(by), cx = bx0 + __builtin_ctz(bx);
                    consider(s, ((ct * s.k[2] + cz) * s.k[1] + cy) * s.k[0] + cx, px, py, pz, pt, v, field, wv,
                             best_d, best);
                }
    return best == 0x7FFFFFFF ? prev : best;
}

// The same search over reach ranges of any width (the slab test inline).
__device__ __noinline__ int assign_wide(const DevS& s, float px, float py, float pz, float pt, float v,
                                        bool field, int prev) {
    const float p[4] = {px, py, pz, pt};
    int lo[4], hi[4];
    for (int d = 0; d < 4; ++d) {
        const int c = seed_cell(p[d], s.C[d], s.k[d]);
        lo[d] = s.reach[(d * s.kmax + c) * 2];
        hi[d] = s.reach[(d * s.kmax + c) * 2 + 1];
    }
    const float wv = field ? s.wf : s.wp;
    float best_d = INFINITY;
    int best = 0x7FFFFFFF;
    for (int ct = lo[3]; ct <= hi[3]; ++ct) {
        if (!slab_holds(s, 3, ct, pt)) continue;
        for (int cz = lo[2]; cz <= hi[2]; ++cz) {
            if (!slab_holds(s, 2, cz, pz)) continue;
            for (int cy = lo[1]; cy <= hi[1]; ++cy) {
                if (!slab_holds(s, 1, cy, py)) continue;
                for (int cx = lo[0]; cx <= hi[0]; ++cx) {
                    if (!slab_holds(s, 0, cx, px)) continue;
                    consider(s, ((ct * s.k[2] + cz) * s.k[1] + cy) * s.k[0] + cx, px, py, pz, pt, v, field, wv,
                             best_d, best);
                }
            }
        }
    }
    return best == 0x7FFFFFFF ? prev : best;
}

__device__ __forceinline__ int assign_one(const DevS& s, float px, float py, float pz, float pt, float v,
                                          bool field, int prev) {
    int b[4];
    bool wide = false;
    const unsigned mx = axis_mask(s, 0, seed_cell(px, s.C[0], s.k[0]), px, b[0], wide);
    const unsigned my = axis_mask(s, 1, seed_cell(py, s.C[1], s.k[1]), py, b[1], wide);
    const unsigned mz = axis_mask(s, 2, seed_cell(pz, s.C[2], s.k[2]), pz, b[2], wide);
    const unsigned mt = axis_mask(s, 3, seed_cell(pt, s.C[3], s.k[3]), pt, b[3], wide);
    if (wide) return assign_wide(s, px, py, pz, pt, v, field, prev);
    return assign_cands(s, px, py, pz, pt, v, field, prev, b[0], b[1], b[2], b[3], mx, my, mz, mt);
}

// Block-local sums keyed by centre id (open addressing).  A sample whose
// centre finds no free slot goes straight to the global sums.
struct Table {
    int key[kTab];
    unsigned long long acc[kTab][kSlicAcc];
};

__device__ __forceinline__ void table_init(Table& tb) {
    for (int i = threadIdx.x; i < kTab * kSlicAcc; i += blockDim.x) (&tb.acc[0][0])[i] = 0ull;
    for (int i = threadIdx.x; i < kTab; i += blockDim.x) tb.key[i] = -1;
    __syncthreads();
}

// One thread's running sums for the centre of its last samples.
struct Run {
    int id;  // -1: none
    long long q[5];
    long long n;
};

__device__ __forceinline__ void add_run(const DevS& s, Table& tb, const Run& r, bool field) {
    if (r.id < 0) return;
    const int id = r.id;
    unsigned long long* dst = nullptr;
    const unsigned h = ((unsigned)id * 2654435761u) >> 26;
    for (int k = 0; k < kTab; ++k) {
        const int slot = (h + k) & (kTab - 1);
        const int was = atomicCAS(&tb.key[slot], -1, id);
        if (was == -1 || was == id) {
            dst = tb.acc[slot];
            break;
        }
    }
    if (!dst) dst = s.acc + (size_t)id * kSlicAcc;  // table full: global (device-scope) atomics
    atomicAdd(&dst[SA_X], (unsigned long long)r.q[0]);
    atomicAdd(&dst[SA_Y], (unsigned long long)r.q[1]);
    atomicAdd(&dst[SA_Z], (unsigned long long)r.q[2]);
    atomicAdd(&dst[SA_T], (unsigned long long)r.q[3]);
    atomicAdd(&dst[field ? SA_F : SA_P], (unsigned long long)r.q[4]);
    atomicAdd(&dst[field ? SA_NF : SA_NP], (unsigned long long)r.n);
}

// Add one sample to the thread's run; a sample of another centre first adds
// the run to the block's sums.
__device__ __forceinline__ void run_sample(const DevS& s, Table& tb, Run& r, int id, const long long* q,
                                           bool field) {
    if (id != r.id) {
        add_run(s, tb, r, field);
        r.id = id;
        r.n = 0;
        for (int k = 0; k < 5; ++k) r.q[k] = 0;
    }
    for (int k = 0; k < 5; ++k) r.q[k] += q[k];
    ++r.n;
}

__device__ __forceinline__ void table_flush(const DevS& s, Table& tb) {
    __syncthreads();
    for (int i = threadIdx.x; i < kTab * kSlicAcc; i += blockDim.x) {
        const int slot = i / kSlicAcc, a = i % kSlicAcc;
        const int id = tb.key[slot];
        const unsigned long long v = tb.acc[slot][a];
        if (id >= 0 && v) atomicAdd(&s.acc[(size_t)id * kSlicAcc + a], v);
    }
}

// Field samples: block b takes samples [b * 1024, (b + 1) * 1024) in
// [T][Z][Y][X] order, 4 consecutive ones per thread (mostly of one centre:
// the thread sums them before touching the block's table).  assign = 0:
// labels from the seed cells.
__global__ __launch_bounds__(kBlock) void k_slic_field(DevS s, int assign) {
    __shared__ Table tb;
    table_init(tb);
    const uint32_t V = (uint32_t)s.X * s.Y * s.Z * s.T;  // < 2^31 (checked by the host)
    const uint32_t i0 = blockIdx.x * (uint32_t)(kBlock * kPer) + threadIdx.x * kPer;
    Run run;
    run.id = -1;
    // coordinates of the thread's first sample (32-bit arithmetic), then
    // stepped along x; what depends only on (y, z, t) is computed per row
    int x = 0, y = 0, z = 0, t = 0;
    if (i0 < V) {
        uint32_t r = i0;
        x = (int)(r % (uint32_t)s.X);
        r /= (uint32_t)s.X;
        y = (int)(r % (uint32_t)s.Y);
        r /= (uint32_t)s.Y;
        z = (int)(r % (uint32_t)s.Z);
        t = (int)(r / (uint32_t)s.Z);
    }
    float py = 0.f, pz = 0.f, pt = 0.f;
    int cy0 = 0, cz0 = 0, ct0 = 0;
    int by0 = 0, bz0 = 0, bt0 = 0;
    unsigned my = 0, mz = 0, mt = 0;
    bool row = false;       // row values current
    bool row_wide = false;  // a reach range of the row wider than 32 slabs
    for (int j = 0; j < kPer; ++j) {
        const uint32_t i = i0 + j;
        if (i >= V) break;
        if (j > 0 && ++x == s.X) {  // next row
            x = 0;
            row = false;
            if (++y == s.Y) {
                y = 0;
                if (++z == s.Z) {
                    z = 0;
                    ++t;
                }
            }
        }
        const float v = s.field[i];
        if (!isfinite(v)) {
            s.labels[i] = -1;
            continue;
        }
        if (!(fabsf(v) < kMaxAbs)) s.counters[SC_RANGE] = 1u;
        if (!row) {
            py = (float)y + 0.5f;
            pz = (float)z + 0.5f;
            pt = (float)t;
            cy0 = seed_cell(py, s.C[1], s.k[1]);
            cz0 = seed_cell(pz, s.C[2], s.k[2]);
            ct0 = seed_cell(pt, s.C[3], s.k[3]);
            if (assign) {
                row_wide = false;
                my = axis_mask(s, 1, cy0, py, by0, row_wide);
                mz = axis_mask(s, 2, cz0, pz, bz0, row_wide);
                mt = axis_mask(s, 3, ct0, pt, bt0, row_wide);
            }
            row = true;
        }
        const float px = (float)x + 0.5f;
        const int cx0 = seed_cell(px, s.C[0], s.k[0]);
        int id;
        if (assign) {
            int bx0;
            bool wide = row_wide;
            const unsigned mx = axis_mask(s, 0, cx0, px, bx0, wide);
            id = wide ? assign_wide(s, px, py, pz, pt, v, true, s.labels[i])
                      : assign_cands(s, px, py, pz, pt, v, true, s.labels[i], bx0, by0, bz0, bt0, mx, my, mz,
                                     mt);
        } else {
            id = ((ct0 * s.k[2] + cz0) * s.k[1] + cy0) * s.k[0] + cx0;
        }
        s.labels[i] = id;
        const long long q[5] = {quantise(px), quantise(py), quantise(pz), (long long)t << 20, quantise(v)};
        run_sample(s, tb, run, id, q, true);
    }
    add_run(s, tb, run, true);
    table_flush(s, tb);
}

// Point samples in visiting order (particle-steps sorted by the tile holding
// them, so that a block meets few centres, with positions, times and values
// copied in that order): block b takes positions [b * 1024, (b + 1) * 1024),
// 4 consecutive ones per thread.  Their labels follow the field's, in the
// same order.
__global__ __launch_bounds__(kBlock) void k_slic_points(DevS s, int assign) {
    __shared__ Table tb;
    table_init(tb);
    const uint64_t V = (uint64_t)s.X * s.Y * s.Z * s.T;
    const uint64_t Q = (uint64_t)s.Tp * s.P;
    const uint64_t base = (uint64_t)blockIdx.x * (kBlock * kPer) + (uint64_t)threadIdx.x * kPer;
    Run run;
    run.id = -1;
    for (int j = 0; j < kPer; ++j) {
        const uint64_t o = base + j;
        if (o >= Q) break;
        const float4 pp = s.spos[o];
        const float v = s.sattr[o];
        const float px = pp.x, py = pp.y, pz = pp.z, pt = pp.w;
        int32_t* lab = s.labels + V + o;
        if (!(isfinite(v) && isfinite(px) && isfinite(py) && isfinite(pz))) {
            *lab = -1;
            continue;
        }
        if (!(fabsf(v) < kMaxAbs && fabsf(px) < kMaxAbs && fabsf(py) < kMaxAbs && fabsf(pz) < kMaxAbs))
            s.counters[SC_RANGE] = 1u;
        int id;
        if (assign) {
            id = assign_one(s, px, py, pz, pt, v, false, *lab);
        } else {
            const int cx = seed_cell(px, s.C[0], s.k[0]), cy = seed_cell(py, s.C[1], s.k[1]);
            const int cz = seed_cell(pz, s.C[2], s.k[2]), ct = seed_cell(pt, s.C[3], s.k[3]);
            id = ((ct * s.k[2] + cz) * s.k[1] + cy) * s.k[0] + cx;
        }
        *lab = id;
        const long long q[5] = {quantise(px), quantise(py), quantise(pz), quantise(pt), quantise(v)};
        run_sample(s, tb, run, id, q, false);
    }
    add_run(s, tb, run, false);
    table_flush(s, tb);
}

// One thread per centre.  seed: write the seed centre first (its location
// ((i + 0.5) C_d), values 0).  Then the means of the sums (a centre without
// samples, or without samples of one type, keeps the previous values), the
// convergence test against the previous centre, and the sums cleared.
__global__ __launch_bounds__(256) void k_slic_update(DevS s, int seed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool moved = false;
    if (i < s.K) {
        double* c = s.cen + (size_t)i * 6;
        if (seed) {
            int r = i;
            const int cx = r % s.k[0];
            r /= s.k[0];
            const int cy = r % s.k[1];
            r /= s.k[1];
            const int cz = r % s.k[2];
            const int ct = r / s.k[2];
            c[0] = (double)__fmul_rn((float)cx + 0.5f, s.C[0]);
            c[1] = (double)__fmul_rn((float)cy + 0.5f, s.C[1]);
            c[2] = (double)__fmul_rn((float)cz + 0.5f, s.C[2]);
            c[3] = (double)__fmul_rn((float)ct + 0.5f, s.C[3]);
            c[4] = 0.0;
            c[5] = 0.0;
        }
        unsigned long long* a = s.acc + (size_t)i * kSlicAcc;
        long long sum[kSlicAcc];
#pragma unroll
        for (int j = 0; j < kSlicAcc; ++j) {
            sum[j] = (long long)a[j];
            s.lsum[(size_t)i * kSlicAcc + j] = a[j];  // kept for the features (Section 3.3)
            a[j] = 0ull;
        }
        const long long nf = sum[SA_NF], np = sum[SA_NP], n = nf + np;
        double nw[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) nw[j] = c[j];
        if (n > 0)
            for (int j = 0; j < 4; ++j) nw[j] = __ddiv_rn(to_double(sum[SA_X + j]), (double)n) * kQInv;
        if (np > 0) nw[4] = __ddiv_rn(to_double(sum[SA_P]), (double)np) * kQInv;
        if (nf > 0) nw[5] = __ddiv_rn(to_double(sum[SA_F]), (double)nf) * kQInv;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if (fabs(__dsub_rn(nw[j], c[j])) > __dmul_rn(s.eps, fabs(c[j]))) moved = true;
            c[j] = nw[j];
            s.cen32[(size_t)i * 8 + j] = (float)nw[j];
        }
        s.cnt[(size_t)i * 2] = nf;
        s.cnt[(size_t)i * 2 + 1] = np;
        // slab bounds of the new centre, on each axis (from the fp32 copy the
        // assignment compares with)
        int r = i;
        for (int d = 0; d < 4; ++d) {
            const int cell = d < 3 ? r % s.k[d] : r;
            r /= s.k[d];
            const uint32_t key = float_key((float)nw[d]);
            atomicMin(&s.slab[(0 * 4 + d) * s.kmax + cell], key);
            atomicMax(&s.slab[(1 * 4 + d) * s.kmax + cell], key);
        }
    }
    const unsigned long long m = __ballot(moved);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&s.counters[SC_MOVED], (unsigned)__popcll(m));
}

inline unsigned blocks_for(uint64_t n, uint64_t per) { return (unsigned)((n + per - 1) / per); }

// ---- cluster merging and feature statistics (Section 3.3) ------------------
//
// Centres i < j match when, per sample type, neither has samples of it or
// both do and their means differ by at most eps * max(|a|, |b|); centres
// without samples match nothing.  Features are the connected components of
// "match" (a lock-free union-find: a root is only ever linked to a smaller
// root, so every component ends rooted at its lowest centre id, whatever the
// order of the unions).  Per feature: exact means from the integer sums of
// its centres, extents and squared deviations from one pass over the samples
// keyed by centre (spatially coherent, like the clustering passes), folded
// into the features.

// Links are read with agent-scope atomic loads: a stale cached link could
// keep a compare-and-swap loop failing.
__device__ __forceinline__ int load_link(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of i, halving the path on the way (i's link moves to its grandparent:
// still an ancestor, and only a non-root's link moves, which no union
// touches).  Links strictly decrease, so the walk is at most K steps (the
// bound only guards against the impossible).
__device__ __forceinline__ int find_root(int* parent, int i, int K) {
    for (int k = 0; k <= K; ++k) {
        const int p = load_link(&parent[i]);
        if (p == i) return i;
        const int gp = load_link(&parent[p]);
        if (gp != p) __hip_atomic_store(&parent[i], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        i = gp;
    }
    return -1;
}

__device__ bool unite(int* parent, int i, int j, int K) {
    for (int k = 0; k <= K + 1; ++k) {  // every failed swap means another union succeeded
        int a = find_root(parent, i, K), b = find_root(parent, j, K);
        if (a < 0 || b < 0) return false;
        if (a == b) return true;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&parent[b], b, a) == b) return true;
    }
    return false;
}

__device__ __forceinline__ bool has_samples(const DevS& s, int i) {
    return s.cnt[2 * (size_t)i] + s.cnt[2 * (size_t)i + 1] > 0;
}

__global__ __launch_bounds__(256) void k_merge_init(DevS s, DevM m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.K) return;
    m.parent[i] = i;
    for (int d = 0; d < 8; ++d) {
        m.cext[8 * (size_t)i + d] = d < 4 ? 0xFFFFFFFFu : 0u;
        m.fext[8 * (size_t)i + d] = d < 4 ? 0xFFFFFFFFu : 0u;
        m.fsum[8 * (size_t)i + d] = 0ull;
    }
    for (int t = 0; t < 2; ++t) {
        m.css[2 * (size_t)i + t] = 0.0;
        m.fss[2 * (size_t)i + t] = 0.0;
    }
}

// Pair tests in tiles of 256 x 256 centres, so that every block does the same
// work (K^2 / 2 tests in all): block (bx, by >= bx) compares the centres of
// tile bx, one per thread, with the later centres of tile by, held in LDS.  Two
// centres match when they have the same sample types and, per type, means
// within eps of the larger magnitude (Section 3.3).
constexpr int kMergeTile = 256;
__global__ __launch_bounds__(kMergeTile) void k_merge_pairs(DevS s, DevM m) {
    if (blockIdx.y < blockIdx.x) return;  // block-uniform: lower triangle
    __shared__ double sv[2][kMergeTile];  // field mean, point mean
    __shared__ unsigned sh[kMergeTile];   // bit 0: has field samples, bit 1: has point samples
    const int j0 = blockIdx.y * kMergeTile;
    {
        const int j = j0 + threadIdx.x;
        unsigned h = 0;
        double vf = 0.0, vp = 0.0;
        if (j < m.K) {
            h = (s.cnt[2 * (size_t)j] > 0 ? 1u : 0u) | (s.cnt[2 * (size_t)j + 1] > 0 ? 2u : 0u);
            vf = s.cen[6 * (size_t)j + 5];
            vp = s.cen[6 * (size_t)j + 4];
        }
        sh[threadIdx.x] = h;
        sv[0][threadIdx.x] = vf;
        sv[1][threadIdx.x] = vp;
    }
    __syncthreads();
    const int i = blockIdx.x * kMergeTile + threadIdx.x;
    if (i >= m.K) return;
    const unsigned hi = (s.cnt[2 * (size_t)i] > 0 ? 1u : 0u) | (s.cnt[2 * (size_t)i + 1] > 0 ? 2u : 0u);
    if (!hi) return;  // no samples: merges with nothing
    const double af = s.cen[6 * (size_t)i + 5], ap = s.cen[6 * (size_t)i + 4];
    const int jn = min(kMergeTile, m.K - j0);
    for (int jj = 0; jj < jn; ++jj) {
        const int j = j0 + jj;
        if (j <= i || sh[jj] != hi) continue;  // a type only one has: different phenomena
        bool ok = true;
        if (hi & 1u) {
            const double b = sv[0][jj];
            ok = fabs(__dsub_rn(af, b)) <= __dmul_rn(m.eps, fmax(fabs(af), fabs(b)));
        }
        if (ok && (hi & 2u)) {
            const double b = sv[1][jj];
            ok = fabs(__dsub_rn(ap, b)) <= __dmul_rn(m.eps, fmax(fabs(ap), fabs(b)));
        }
        if (ok && !unite(m.parent, i, j, m.K)) m.err[0] = 1u;
    }
}

__global__ __launch_bounds__(256) void k_merge_flatten(DevS s, DevM m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.K) return;
    int f = -1;
    if (has_samples(s, i)) {
        f = find_root(m.parent, i, m.K);
        if (f < 0) m.err[0] = 1u;
    }
    m.feat[i] = f;
}

// The lanes of a wave that hold centres of one feature combine their values
// first, so that one lane per (wave, feature) updates the feature (most
// centres of a wave usually share one).  Visits each distinct feature of the
// wave in turn: fn(feature, this lane holds it, this lane updates it); F < 0:
// no centre.
template <typename Fn>
__device__ __forceinline__ void per_wave_feature(int F, Fn&& fn) {
    unsigned long long pending = __ballot(F >= 0);
    while (pending) {  // wave-uniform
        const int leader = __ffsll((long long)pending) - 1;
        const int FL = __shfl(F, leader);
        const bool mine = F == FL;
        pending &= ~__ballot(mine);
        fn(FL, mine, (int)__lane_id() == leader);
    }
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(256) void k_feature_sums(DevS s, DevM m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int F = i < m.K ? m.feat[i] : -1;
    unsigned long long v[kSlicAcc];
    for (int j = 0; j < kSlicAcc; ++j) v[j] = F >= 0 ? s.lsum[8 * (size_t)i + j] : 0ull;
    per_wave_feature(F, [&](int FL, bool mine, bool lead) {
        for (int j = 0; j < kSlicAcc; ++j) {
            const unsigned long long x = wave_sum_u64(mine ? v[j] : 0ull);
            if (lead) atomicAdd(&m.fsum[8 * (size_t)FL + j], x);
        }
    });
}

__global__ __launch_bounds__(256) void k_feature_means(DevS s, DevM m) {
    const int F = blockIdx.x * blockDim.x + threadIdx.x;
    if (F >= m.K || m.feat[F] != F) return;
    const unsigned long long* a = m.fsum + 8 * (size_t)F;
    const long long nf = (long long)a[SA_NF], np = (long long)a[SA_NP];
    m.fmean[2 * (size_t)F] = nf > 0 ? __ddiv_rn(to_double((long long)a[SA_F]), (double)nf) * kQInv : 0.0;
    m.fmean[2 * (size_t)F + 1] = np > 0 ? __ddiv_rn(to_double((long long)a[SA_P]), (double)np) * kQInv : 0.0;
}

// Block-local extents and squared deviations keyed by centre.
struct StatTable {
    int key[kTab];
    uint32_t ext[kTab][8];
    double ss[kTab];
};

struct StatRun {
    int id;
    uint32_t ext[8];
    double ss;
};

__device__ __forceinline__ void stat_init(StatTable& tb) {
    for (int i = threadIdx.x; i < kTab; i += blockDim.x) {
        tb.key[i] = -1;
        tb.ss[i] = 0.0;
        for (int d = 0; d < 8; ++d) tb.ext[i][d] = d < 4 ? 0xFFFFFFFFu : 0u;
    }
    __syncthreads();
}

__device__ __forceinline__ void stat_add(const DevM& m, StatTable& tb, const StatRun& r, int ty) {
    if (r.id < 0) return;
    uint32_t* ext = nullptr;
    double* ss = nullptr;
    const unsigned h = ((unsigned)r.id * 2654435761u) >> 26;
    for (int k = 0; k < kTab; ++k) {
        const int slot = (h + k) & (kTab - 1);
        const int was = atomicCAS(&tb.key[slot], -1, r.id);
        if (was == -1 || was == r.id) {
            ext = tb.ext[slot];
            ss = &tb.ss[slot];
            break;
        }
    }
    if (!ext) {  // table full: straight to the centre's accumulators
        ext = m.cext + 8 * (size_t)r.id;
        ss = m.css + 2 * (size_t)r.id + ty;
    }
    for (int d = 0; d < 4; ++d) {
        atomicMin(&ext[d], r.ext[d]);
        atomicMax(&ext[4 + d], r.ext[4 + d]);
    }
    atomicAdd(ss, r.ss);
}

__device__ __forceinline__ void stat_sample(const DevM& m, StatTable& tb, StatRun& r, int id, const float* c,
                                            double dev, int ty) {
    if (id != r.id) {
        stat_add(m, tb, r, ty);
        r.id = id;
        r.ss = 0.0;
        for (int d = 0; d < 4; ++d) {
            r.ext[d] = 0xFFFFFFFFu;
            r.ext[4 + d] = 0u;
        }
    }
    for (int d = 0; d < 4; ++d) {
        const uint32_t k = float_key(c[d]);
        r.ext[d] = min(r.ext[d], k);
        r.ext[4 + d] = max(r.ext[4 + d], k);
    }
    r.ss += dev * dev;
}

__device__ __forceinline__ void stat_flush(const DevM& m, StatTable& tb, int ty) {
    __syncthreads();
    for (int slot = threadIdx.x; slot < kTab; slot += blockDim.x) {
        const int id = tb.key[slot];
        if (id < 0) continue;
        for (int d = 0; d < 4; ++d) {
            atomicMin(&m.cext[8 * (size_t)id + d], tb.ext[slot][d]);
            atomicMax(&m.cext[8 * (size_t)id + 4 + d], tb.ext[slot][4 + d]);
        }
        atomicAdd(&m.css[2 * (size_t)id + ty], tb.ss[slot]);
    }
}

// ty 0: field samples [T][Z][Y][X]; ty 1: point samples in visiting order.
__global__ __launch_bounds__(kBlock) void k_feature_pass(DevS s, DevM m, int ty) {
    __shared__ StatTable tb;
    stat_init(tb);
    const uint64_t V = (uint64_t)s.X * s.Y * s.Z * s.T;
    const uint64_t N = ty == 0 ? V : (uint64_t)s.Tp * s.P;
    const uint64_t base = (uint64_t)blockIdx.x * (kBlock * kPer) + (uint64_t)threadIdx.x * kPer;
    StatRun run;
    run.id = -1;
    for (int j = 0; j < kPer; ++j) {
        const uint64_t i = base + j;
        if (i >= N) break;
        const int L = s.labels[(ty == 0 ? 0 : V) + i];
        if (L < 0) continue;
        float c[4], v;
        if (ty == 0) {
            uint32_t r = (uint32_t)i;
            c[0] = (float)(r % (uint32_t)s.X) + 0.5f;
            r /= (uint32_t)s.X;
            c[1] = (float)(r % (uint32_t)s.Y) + 0.5f;
            r /= (uint32_t)s.Y;
            c[2] = (float)(r % (uint32_t)s.Z) + 0.5f;
            c[3] = (float)(r / (uint32_t)s.Z);
            v = s.field[i];
        } else {
            const float4 pp = s.spos[i];
            c[0] = pp.x;
            c[1] = pp.y;
            c[2] = pp.z;
            c[3] = pp.w;
            v = s.sattr[i];
        }
        const double dev = (double)v - m.fmean[2 * (size_t)m.feat[L] + ty];
        stat_sample(m, tb, run, L, c, dev, ty);
    }
    stat_add(m, tb, run, ty);
    stat_flush(m, tb, ty);
}

// Per-centre extents and squared deviations folded into their features, one
// update per (wave, feature).
__global__ __launch_bounds__(256) void k_feature_fold(DevM m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int F = i < m.K ? m.feat[i] : -1;
    uint32_t e[8];
    double q[2];
    for (int d = 0; d < 8; ++d) e[d] = F >= 0 ? m.cext[8 * (size_t)i + d] : (d < 4 ? 0xFFFFFFFFu : 0u);
    for (int t = 0; t < 2; ++t) q[t] = F >= 0 ? m.css[2 * (size_t)i + t] : 0.0;
    per_wave_feature(F, [&](int FL, bool mine, bool lead) {
        for (int d = 0; d < 8; ++d) {
            uint32_t x = mine ? e[d] : (d < 4 ? 0xFFFFFFFFu : 0u);
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t y = __shfl_xor(x, o);
                x = d < 4 ? min(x, y) : max(x, y);
            }
            if (lead) {
                if (d < 4) atomicMin(&m.fext[8 * (size_t)FL + d], x);
                else atomicMax(&m.fext[8 * (size_t)FL + d], x);
            }
        }
        for (int t = 0; t < 2; ++t) {
            double x = mine ? q[t] : 0.0;
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
            if (lead) atomicAdd(&m.fss[2 * (size_t)FL + t], x);
        }
    });
}

__global__ __launch_bounds__(256) void k_feature_write(DevM m) {
    const int F = blockIdx.x * blockDim.x + threadIdx.x;
    if (F >= m.K) return;
    double* o = m.out + (size_t)F * kFeatStats;
    for (int k = 0; k < kFeatStats; ++k) o[k] = 0.0;
    if (m.feat[F] != F) return;
    const unsigned long long* a = m.fsum + 8 * (size_t)F;
    const double nf = (double)(long long)a[SA_NF], np = (double)(long long)a[SA_NP];
    o[FS_NF] = nf;
    o[FS_NP] = np;
    o[FS_MEAN_F] = m.fmean[2 * (size_t)F];
    o[FS_MEAN_P] = m.fmean[2 * (size_t)F + 1];
    o[FS_STD_F] = nf > 0 ? sqrt(m.fss[2 * (size_t)F] / nf) : 0.0;
    o[FS_STD_P] = np > 0 ? sqrt(m.fss[2 * (size_t)F + 1] / np) : 0.0;
    for (int d = 0; d < 4; ++d) {
        o[FS_XMIN + 2 * d] = (double)key_float(m.fext[8 * (size_t)F + d]);
        o[FS_XMIN + 2 * d + 1] = (double)key_float(m.fext[8 * (size_t)F + 4 + d]);
    }
}

// ---- visiting order of the point samples (counting sort by tile) ----------

constexpr uint32_t kSkip = 0xFFFFFFFFu;  // a padding step (t >= T): not a sample
constexpr int kScanBlocks = 1024;

// Sort key of particle-step e = p * Tpad + t.
__device__ __forceinline__ uint32_t order_key(const uint32_t* bins, uint64_t e, uint64_t Qpad, int Tpad,
                                              int T, int shift, uint32_t none) {
    if (e >= Qpad) return kSkip;
    const uint64_t p = e / (uint64_t)Tpad;
    if ((int)(e - p * Tpad) >= T) return kSkip;
    const uint32_t b = bins[e];
    return b == 0xFFFFFFFFu ? none : b >> shift;
}

// A wave holds 64 consecutive steps; consecutive steps of a trajectory mostly
// share a tile, so lanes split into runs of one key and only a run's first
// lane (head) touches the key's counter.
struct KeyRun {
    int head, len;
};

__device__ __forceinline__ KeyRun key_run(uint32_t key) {
    const int lane = threadIdx.x & 63;
    const uint32_t prev = (uint32_t)__shfl_up((int)key, 1);
    const unsigned long long starts = __ballot(lane == 0 || prev != key);
    const unsigned long long later = lane == 63 ? 0ull : starts >> (lane + 1);
    KeyRun r;
    r.len = later ? __builtin_ctzll(later) + 1 : 64 - lane;
    const unsigned long long upto = lane == 63 ? starts : starts & ((2ull << lane) - 1);
    r.head = 63 - __builtin_clzll(upto);  // lane 0 always starts a run
    return r;
}

__global__ __launch_bounds__(256) void k_order_count(const uint32_t* __restrict__ bins, uint64_t Qpad,
                                                     int Tpad, int T, int shift, uint32_t none,
                                                     uint32_t* __restrict__ cnt) {
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t w = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6; w * 64 < Qpad; w += nwaves) {
        const uint32_t key = order_key(bins, w * 64 + (threadIdx.x & 63), Qpad, Tpad, T, shift, none);
        const KeyRun r = key_run(key);
        if (key != kSkip && r.head == (int)(threadIdx.x & 63)) atomicAdd(&cnt[key], (uint32_t)r.len);
    }
}

// Exclusive prefix of the 256 values of a block; `total` gets their sum.
__device__ __forceinline__ uint32_t block_scan256(uint32_t v, uint32_t* s_w, uint32_t& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int i = 0; i < wave; ++i) base += s_w[i];
    total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
    return base + x - v;
}

// Counts -> exclusive offsets, in place, over n buckets: per-block sums of
// consecutive ranges, one block scans them, each block writes its offsets.
__global__ __launch_bounds__(256) void k_order_sums(const uint32_t* __restrict__ cnt, uint32_t n,
                                                    uint32_t* __restrict__ bsum) {
    const uint32_t per = (n + kScanBlocks - 1) / kScanBlocks;
    const uint32_t i0 = blockIdx.x * per, i1 = min(n, i0 + per);
    uint32_t c = 0;
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) c += cnt[i];
    for (int o = 32; o > 0; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o);
    __shared__ uint32_t s_w[4];
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__global__ __launch_bounds__(1024) void k_order_top(uint32_t* __restrict__ bsum) {
    __shared__ uint32_t s_w[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t v = bsum[threadIdx.x];
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int i = 0; i < wave; ++i) base += s_w[i];
    bsum[threadIdx.x] = base + x - v;
}

__global__ __launch_bounds__(256) void k_order_offsets(uint32_t* __restrict__ cnt, uint32_t n,
                                                       const uint32_t* __restrict__ bsum) {
    __shared__ uint32_t s_w[4];
    const uint32_t per = (n + kScanBlocks - 1) / kScanBlocks;
    const uint32_t i0 = blockIdx.x * per, i1 = min(n, i0 + per);
    uint32_t base = bsum[blockIdx.x];
    for (uint32_t b0 = i0; b0 < i1; b0 += blockDim.x) {  // block-uniform
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t v = i < i1 ? cnt[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_scan256(v, s_w, total);
        if (i < i1) cnt[i] = base + ex;
        base += total;
    }
}

__global__ __launch_bounds__(256) void k_order_scatter(const uint32_t* __restrict__ bins, uint64_t Qpad,
                                                       int Tpad, int T, int rate, int shift, uint32_t none, int64_t P,
                                                       uint32_t* __restrict__ cur, uint32_t* __restrict__ order,
                                                       const float* __restrict__ xyz,
                                                       const float* __restrict__ attr,
                                                       float4* __restrict__ spos, float* __restrict__ sattr) {
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const int lane = threadIdx.x & 63;
    for (uint64_t w = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6; w * 64 < Qpad; w += nwaves) {
        const uint64_t e = w * 64 + lane;
        const uint32_t key = order_key(bins, e, Qpad, Tpad, T, shift, none);
        const KeyRun r = key_run(key);
        uint32_t at = 0;
        if (key != kSkip && r.head == lane) at = atomicAdd(&cur[key], (uint32_t)r.len);
        at = (uint32_t)__shfl((int)at, r.head) + (uint32_t)(lane - r.head);
        if (key != kSkip) {
            const uint64_t p = e / (uint64_t)Tpad;
            const uint64_t t = e - p * Tpad;
            const uint64_t i = t * (uint64_t)P + p;
            order[i] = at;  // position of step i in the visiting order
            spos[at] = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], __fdiv_rn((float)t, (float)rate));
            sattr[at] = attr[i];
        }
    }
}

}  // namespace

// Gathers, so that the writes of [T][P] are coalesced: out[q] = in[pos[q]].
__global__ __launch_bounds__(256) void k_slic_unsort(const int32_t* __restrict__ in,
                                                     const uint32_t* __restrict__ pos, uint64_t Q,
                                                     int32_t* __restrict__ out) {
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < Q; q += (uint64_t)gridDim.x * blockDim.x)
        out[q] = in[pos[q]];
}

// Trajectory segments of the features (Section 3.4): a particle-step keeps
// its feature id when the same particle lies in that feature at t - 1 or
// t + 1 (so that runs of two or more consecutive steps are drawn), else -1.
// In place on point labels [T][P]: a thread owns one particle and reads its
// step t + 1 before it writes step t.  feat[centre] -> feature id.
__global__ __launch_bounds__(256) void k_slic_segments(int32_t* __restrict__ lab, const int32_t* __restrict__ feat,
                                                      int T, int64_t P) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += stride) {
        auto fid = [&](int t) -> int32_t {
            const int32_t l = lab[(int64_t)t * P + p];
            return l >= 0 ? feat[l] : -1;
        };
        int32_t prev = -1, cur = fid(0);
        for (int t = 0; t < T; ++t) {
            const int32_t next = t + 1 < T ? fid(t + 1) : -1;
            lab[(int64_t)t * P + p] = cur >= 0 && (cur == prev || cur == next) ? cur : -1;
            prev = cur;
            cur = next;
        }
    }
}

void launch_slic_segments(int32_t* lab, const int32_t* feat, int T, int64_t P, hipStream_t st) {
    if (T <= 0 || P <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>((P + 255) / 256, 16384);
    hipLaunchKernelGGL(k_slic_segments, dim3(g), dim3(256), 0, st, lab, feat, T, P);
}

void launch_slic_unsort(const int32_t* in, const uint32_t* order, uint64_t Q, int32_t* out, hipStream_t st) {
    if (Q == 0) return;
    const unsigned g = (unsigned)std::min<uint64_t>((Q + 255) / 256, 16384);
    hipLaunchKernelGGL(k_slic_unsort, dim3(g), dim3(256), 0, st, in, order, Q, out);
}

int launch_slic_order(const uint32_t* bins, const float* xyz, const float* attr, int64_t P, int Tpad,
                      int T, int r, int shift, uint32_t ntiles, uint32_t* scratch, uint32_t* order, float4* spos,
                      float* sattr, hipStream_t st) {
    const uint64_t Qpad = (uint64_t)P * Tpad;
    const uint32_t nb = ntiles + 1;  // the last bucket: steps in no voxel
    uint32_t* cnt = scratch;
    uint32_t* bsum = scratch + nb + 1;
    if (hipMemsetAsync(cnt, 0, (size_t)nb * sizeof(uint32_t), st) != hipSuccess) return (int)hipGetLastError();
    const unsigned g = (unsigned)std::min<uint64_t>((Qpad + 255) / 256, 8192);
    hipLaunchKernelGGL(k_order_count, dim3(g), dim3(256), 0, st, bins, Qpad, Tpad, T, shift, ntiles, cnt);
    hipLaunchKernelGGL(k_order_sums, dim3(kScanBlocks), dim3(256), 0, st, cnt, nb, bsum);
    hipLaunchKernelGGL(k_order_top, dim3(1), dim3(kScanBlocks), 0, st, bsum);
    hipLaunchKernelGGL(k_order_offsets, dim3(kScanBlocks), dim3(256), 0, st, cnt, nb, bsum);
    hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, st, bins, Qpad, Tpad, T, r, shift, ntiles, P, cnt,
                       order, xyz, attr, spos, sattr);
    return (int)hipGetLastError();
}

void launch_slic_init(const DevS& s, hipStream_t st) {
    const uint64_t V = (uint64_t)s.X * s.Y * s.Z * s.T, Q = (uint64_t)s.Tp * s.P;
    if (V) hipLaunchKernelGGL(k_slic_field, dim3(blocks_for(V, kBlock * kPer)), dim3(kBlock), 0, st, s, 0);
    if (Q) hipLaunchKernelGGL(k_slic_points, dim3(blocks_for(Q, kBlock * kPer)), dim3(kBlock), 0, st, s, 0);
}

void launch_slic_assign(const DevS& s, hipStream_t st) {
    const uint64_t V = (uint64_t)s.X * s.Y * s.Z * s.T, Q = (uint64_t)s.Tp * s.P;
    if (V) hipLaunchKernelGGL(k_slic_field, dim3(blocks_for(V, kBlock * kPer)), dim3(kBlock), 0, st, s, 1);
    if (Q) hipLaunchKernelGGL(k_slic_points, dim3(blocks_for(Q, kBlock * kPer)), dim3(kBlock), 0, st, s, 1);
}

__global__ void k_slic_slab_reset(DevS s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 8 * s.kmax) {
        s.slab[i] = i < 4 * s.kmax ? 0xFFFFFFFFu : 0u;
        s.reach[i] = (i & 1) ? -1 : 0x7FFFFFFF;
    }
}

// Slab i of axis d (bounds lo, hi from the update) can hold a centre within
// C of any p in [lo - C, hi + C], widened by C 2^-20 for the rounding of the
// window test's difference.  Those p fall in the seed cells from floor of
// the lower end / C to floor of the upper end / C (clamped like seed_cell),
// widened by 10^-3 of a cell for the rounding of the division (below 2.5e-4
// of a cell wherever the cell index is below 4096).  Each of those cells
// takes i into its reach range.
__global__ void k_slic_reach(DevS s) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int d = g / s.kmax, i = g - d * s.kmax;
    if (d >= 4 || i >= s.k[d]) return;
    const double C = s.C[d];
    const double lo = key_float(s.slab[(0 * 4 + d) * s.kmax + i]);
    const double hi = key_float(s.slab[(1 * 4 + d) * s.kmax + i]);
    const double m = C * (1.0 + 0x1p-20);
    const double kd = s.k[d] - 1;
    const int j0 = (int)fmin(fmax(floor((lo - m) / C - 1e-3), 0.0), kd);
    const int j1 = (int)fmin(fmax(floor((hi + m) / C + 1e-3), 0.0), kd);
    for (int j = j0; j <= j1; ++j) {
        atomicMin(&s.reach[(d * s.kmax + j) * 2], i);
        atomicMax(&s.reach[(d * s.kmax + j) * 2 + 1], i);
    }
}

void launch_slic_update(const DevS& s, int seed, hipStream_t st) {
    hipLaunchKernelGGL(k_slic_slab_reset, dim3(blocks_for((uint64_t)8 * s.kmax, 256)), dim3(256), 0, st, s);
    hipLaunchKernelGGL(k_slic_update, dim3(blocks_for((uint64_t)s.K, 256)), dim3(256), 0, st, s, seed);
    hipLaunchKernelGGL(k_slic_reach, dim3(blocks_for((uint64_t)4 * s.kmax, 256)), dim3(256), 0, st, s);
}

int launch_slic_merge(const DevS& s, const DevM& m, hipStream_t st) {
    const dim3 gk(blocks_for((uint64_t)m.K, 256)), b256(256);
    const uint64_t V = (uint64_t)s.X * s.Y * s.Z * s.T, Q = (uint64_t)s.Tp * s.P;
    hipLaunchKernelGGL(k_merge_init, gk, b256, 0, st, s, m);
    const unsigned nt = (unsigned)((m.K + kMergeTile - 1) / kMergeTile);
    hipLaunchKernelGGL(k_merge_pairs, dim3(nt, nt), dim3(kMergeTile), 0, st, s, m);
    hipLaunchKernelGGL(k_merge_flatten, gk, b256, 0, st, s, m);
    hipLaunchKernelGGL(k_feature_sums, gk, b256, 0, st, s, m);
    hipLaunchKernelGGL(k_feature_means, gk, b256, 0, st, s, m);
    if (V) hipLaunchKernelGGL(k_feature_pass, dim3(blocks_for(V, kBlock * kPer)), dim3(kBlock), 0, st, s, m, 0);
    if (Q) hipLaunchKernelGGL(k_feature_pass, dim3(blocks_for(Q, kBlock * kPer)), dim3(kBlock), 0, st, s, m, 1);
    hipLaunchKernelGGL(k_feature_fold, gk, b256, 0, st, m);
    hipLaunchKernelGGL(k_feature_write, gk, b256, 0, st, m);
    return (int)hipGetLastError();
}

}  // namespace mf4d
