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

// Centre with the smallest distance among those seeded in the 3^4 cells
// around the sample's seed cell whose window holds the sample; ties go to the
// lowest id; none: `prev`.
__device__ int assign_one(const DevS& s, float px, float py, float pz, float pt, float v, bool field,
                          int prev) {
    const int cx0 = seed_cell(px, s.C[0], s.k[0]), cy0 = seed_cell(py, s.C[1], s.k[1]);
    const int cz0 = seed_cell(pz, s.C[2], s.k[2]), ct0 = seed_cell(pt, s.C[3], s.k[3]);
    const float wv = field ? s.wf : s.wp;
    float best_d = INFINITY;
    int best = 0x7FFFFFFF;
    for (int ct = max(ct0 - 1, 0); ct <= min(ct0 + 1, s.k[3] - 1); ++ct)
        for (int cz = max(cz0 - 1, 0); cz <= min(cz0 + 1, s.k[2] - 1); ++cz)
            for (int cy = max(cy0 - 1, 0); cy <= min(cy0 + 1, s.k[1] - 1); ++cy)
                for (int cx = max(cx0 - 1, 0); cx <= min(cx0 + 1, s.k[0] - 1); ++cx) {
                    const int id = ((ct * s.k[2] + cz) * s.k[1] + cy) * s.k[0] + cx;
                    const float4 c = reinterpret_cast<const float4*>(s.cen32)[2 * id];
                    const float2 cv = reinterpret_cast<const float2*>(s.cen32)[4 * id + 2];
                    const float dx = __fsub_rn(px, c.x), dy = __fsub_rn(py, c.y);
                    const float dz = __fsub_rn(pz, c.z), dt = __fsub_rn(pt, c.w);
                    if (!(fabsf(dx) <= s.C[0] && fabsf(dy) <= s.C[1] && fabsf(dz) <= s.C[2] &&
                          fabsf(dt) <= s.C[3]))
                        continue;
                    const float ctd = __fmul_rn(s.cf, dt);
                    const float sq = __fadd_rn(
                        __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz)),
                        __fmul_rn(ctd, ctd));
                    const float S = __fsqrt_rn(sq);
                    const float vc = field ? cv.y : cv.x;
                    const float D = __fadd_rn(__fmul_rn(wv, fabsf(__fsub_rn(v, vc))), __fmul_rn(s.wd, S));
                    if (D < best_d || (D == best_d && id < best)) {
                        best_d = D;
                        best = id;
                    }
                }
    return best == 0x7FFFFFFF ? prev : best;
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

__device__ __forceinline__ void add_sample(const DevS& s, Table& tb, int id, const long long* q,
                                           bool field) {
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
    atomicAdd(&dst[SA_X], (unsigned long long)q[0]);
    atomicAdd(&dst[SA_Y], (unsigned long long)q[1]);
    atomicAdd(&dst[SA_Z], (unsigned long long)q[2]);
    atomicAdd(&dst[SA_T], (unsigned long long)q[3]);
    atomicAdd(&dst[field ? SA_F : SA_P], (unsigned long long)q[4]);
    atomicAdd(&dst[field ? SA_NF : SA_NP], 1ull);
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
// [T][Z][Y][X] order.  assign = 0: labels from the seed cells.
__global__ __launch_bounds__(kBlock) void k_slic_field(DevS s, int assign) {
    __shared__ Table tb;
    table_init(tb);
    const uint64_t V = (uint64_t)s.X * s.Y * s.Z * s.T;
    const uint64_t base = (uint64_t)blockIdx.x * (kBlock * kPer);
    for (int j = 0; j < kPer; ++j) {
        const uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
        if (i >= V) break;
        const float v = s.field[i];
        if (!isfinite(v)) {
            s.labels[i] = -1;
            continue;
        }
        if (!(fabsf(v) < kMaxAbs)) s.counters[SC_RANGE] = 1u;
        uint64_t r = i;
        const int x = (int)(r % s.X);
        r /= s.X;
        const int y = (int)(r % s.Y);
        r /= s.Y;
        const int z = (int)(r % s.Z);
        const int t = (int)(r / s.Z);
        const float px = (float)x + 0.5f, py = (float)y + 0.5f, pz = (float)z + 0.5f, pt = (float)t;
        int id;
        if (assign) {
            id = assign_one(s, px, py, pz, pt, v, true, s.labels[i]);
        } else {
            const int cx = seed_cell(px, s.C[0], s.k[0]), cy = seed_cell(py, s.C[1], s.k[1]);
            const int cz = seed_cell(pz, s.C[2], s.k[2]), ct = seed_cell(pt, s.C[3], s.k[3]);
            id = ((ct * s.k[2] + cz) * s.k[1] + cy) * s.k[0] + cx;
        }
        s.labels[i] = id;
        const long long q[5] = {quantise(px), quantise(py), quantise(pz), (long long)t << 20, quantise(v)};
        add_sample(s, tb, id, q, true);
    }
    table_flush(s, tb);
}

// Point samples: block b takes particle-steps [b * 1024, (b + 1) * 1024) in
// [T][P] order; their labels follow the field's.
__global__ __launch_bounds__(kBlock) void k_slic_points(DevS s, int assign) {
    __shared__ Table tb;
    table_init(tb);
    const uint64_t V = (uint64_t)s.X * s.Y * s.Z * s.T;
    const uint64_t Q = (uint64_t)s.T * s.P;
    const uint64_t base = (uint64_t)blockIdx.x * (kBlock * kPer);
    for (int j = 0; j < kPer; ++j) {
        const uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
        if (i >= Q) break;
        const float v = s.attr[i];
        const float px = s.xyz[3 * i], py = s.xyz[3 * i + 1], pz = s.xyz[3 * i + 2];
        int32_t* lab = s.labels + V + i;
        if (!(isfinite(v) && isfinite(px) && isfinite(py) && isfinite(pz))) {
            *lab = -1;
            continue;
        }
        if (!(fabsf(v) < kMaxAbs && fabsf(px) < kMaxAbs && fabsf(py) < kMaxAbs && fabsf(pz) < kMaxAbs))
            s.counters[SC_RANGE] = 1u;
        const int t = (int)(i / (uint64_t)s.P);
        const float pt = (float)t;
        int id;
        if (assign) {
            id = assign_one(s, px, py, pz, pt, v, false, *lab);
        } else {
            const int cx = seed_cell(px, s.C[0], s.k[0]), cy = seed_cell(py, s.C[1], s.k[1]);
            const int cz = seed_cell(pz, s.C[2], s.k[2]), ct = seed_cell(pt, s.C[3], s.k[3]);
            id = ((ct * s.k[2] + cz) * s.k[1] + cy) * s.k[0] + cx;
        }
        *lab = id;
        const long long q[5] = {quantise(px), quantise(py), quantise(pz), (long long)t << 20, quantise(v)};
        add_sample(s, tb, id, q, false);
    }
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
    }
    const unsigned long long m = __ballot(moved);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&s.counters[SC_MOVED], (unsigned)__popcll(m));
}

inline unsigned blocks_for(uint64_t n, uint64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void launch_slic_init(const DevS& s, hipStream_t st) {
    const uint64_t V = (uint64_t)s.X * s.Y * s.Z * s.T, Q = (uint64_t)s.T * s.P;
    if (V) hipLaunchKernelGGL(k_slic_field, dim3(blocks_for(V, kBlock * kPer)), dim3(kBlock), 0, st, s, 0);
    if (Q) hipLaunchKernelGGL(k_slic_points, dim3(blocks_for(Q, kBlock * kPer)), dim3(kBlock), 0, st, s, 0);
}

void launch_slic_assign(const DevS& s, hipStream_t st) {
    const uint64_t V = (uint64_t)s.X * s.Y * s.Z * s.T, Q = (uint64_t)s.T * s.P;
    if (V) hipLaunchKernelGGL(k_slic_field, dim3(blocks_for(V, kBlock * kPer)), dim3(kBlock), 0, st, s, 1);
    if (Q) hipLaunchKernelGGL(k_slic_points, dim3(blocks_for(Q, kBlock * kPer)), dim3(kBlock), 0, st, s, 1);
}

void launch_slic_update(const DevS& s, int seed, hipStream_t st) {
    hipLaunchKernelGGL(k_slic_update, dim3(blocks_for((uint64_t)s.K, 256)), dim3(256), 0, st, s, seed);
}

}  // namespace mf4d
