// Brick-activity predictor: a 3-layer 3D convolutional network over the grid of
// 8^3-voxel bricks of each timestep, trained on the grower's own results and
// used to choose which candidate tiles get their admissibility tested before
// the rounds start (the rest are tested when a sweep first reaches them).
//
// Activations are channels-last bf16 [N][D][H][W][16] (unused channels zero);
// every layer is a 16 -> 16 channel 3x3x3 convolution with zero padding, run
// as 27 accumulated v_mfma_f32_16x16x16_bf16 per tile of 16 positions along x
// (fp32 accumulation).  The input-gradient of a layer is the same convolution
// with transposed, point-reflected weights; the weight gradient is a reduction
// over positions on the same matrix cores, per block, then summed in a fixed
// order (deterministic).  Parameters are fp32 masters updated by Adam.
#include "nn.h"

namespace mf4d {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// fp32 -> bf16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int TX = 16, TY = 4, TZ = 4;                  // output positions per block
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;   // with halo
constexpr int kTilePos = TX * TY * TZ;                 // 256

struct ConvDims {
    int N, D, H, W;
    int nbx, nby, nbz;  // blocks per axis
};

__device__ __forceinline__ void block_origin(const ConvDims& c, uint32_t blk, int& n, int& z0,
                                             int& y0, int& x0) {
    x0 = (blk % c.nbx) * TX;
    blk /= c.nbx;
    y0 = (blk % c.nby) * TY;
    blk /= c.nby;
    z0 = (blk % c.nbz) * TZ;
    n = blk / c.nbz;
}

// Stage a (TZ+2)(TY+2)(TX+2) x 16-channel bf16 input tile (zero outside).
__device__ void load_halo(const ConvDims& c, const uint16_t* __restrict__ x, int n, int z0, int y0,
                          int x0, uint16_t* s_x) {
    for (int p = threadIdx.x; p < HZ * HY * HX; p += blockDim.x) {
        const int hx = p % HX, hy = (p / HX) % HY, hz = p / (HX * HY);
        const int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
        uint4 lo = make_uint4(0, 0, 0, 0), hi = make_uint4(0, 0, 0, 0);
        if (zz >= 0 && zz < c.D && yy >= 0 && yy < c.H && xx >= 0 && xx < c.W) {
            const uint4* src = reinterpret_cast<const uint4*>(
                x + ((((size_t)n * c.D + zz) * c.H + yy) * c.W + xx) * 16);
            lo = src[0];
            hi = src[1];
        }
        uint4* dst = reinterpret_cast<uint4*>(s_x + (size_t)p * 16);
        dst[0] = lo;
        dst[1] = hi;
    }
}

// out = conv(x, w) + bias, optionally ReLU, optionally times (mask > 0).
// w: bf16 [27][16 out][16 in].  Writes bf16 [..][16] or, with out_f32, the
// first channel as fp32 [N][D][H][W].
__global__ __launch_bounds__(256) void k_conv16(ConvDims c, const uint16_t* __restrict__ x,
                                                const uint16_t* __restrict__ w,
                                                const float* __restrict__ bias, int relu,
                                                const uint16_t* __restrict__ mask,
                                                uint16_t* __restrict__ out_bf, float* __restrict__ out_f32,
                                                int f32_all) {
    __shared__ uint16_t s_x[HZ * HY * HX * 16];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    // B operand for every offset: W[k][out = row][in = 4*grp .. 4*grp+3]
    v4s bw[27];
#pragma unroll
    for (int k = 0; k < 27; ++k)
        bw[k] = *reinterpret_cast<const v4s*>(w + ((size_t)k * 16 + row) * 16 + 4 * grp);
    const float b = bias ? bias[row] : 0.0f;
    const uint32_t nblocks = (uint32_t)c.N * c.nbz * c.nby * c.nbx;
    for (uint32_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        int n, z0, y0, x0;
        block_origin(c, blk, n, z0, y0, x0);
        __syncthreads();
        load_halo(c, x, n, z0, y0, x0, s_x);
        __syncthreads();
        for (int r = wave; r < TZ * TY; r += 4) {
            const int zl = r / TY, yl = r % TY;
            v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int k = 0; k < 27; ++k) {
                const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
                // A operand: positions x0 + row (+dx), channels 4*grp..4*grp+3
                const uint16_t* src =
                    s_x + (((size_t)(zl + 1 + dz) * HY + (yl + 1 + dy)) * HX + (row + 1 + dx)) * 16 + 4 * grp;
                const v4s a = *reinterpret_cast<const v4s*>(src);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[k], acc, 0, 0, 0);
            }
            // acc[i] = D[pos = 4*grp + i][out channel = row]
            const int z = z0 + zl, y = y0 + yl;
            if (z >= c.D || y >= c.H) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int xx = x0 + 4 * grp + i;
                if (xx >= c.W) continue;
                const size_t pos = (((size_t)n * c.D + z) * c.H + y) * c.W + xx;
                float v = acc[i] + b;
                if (relu) v = fmaxf(v, 0.0f);
                if (mask && !(bf2f(mask[pos * 16 + row]) > 0.0f)) v = 0.0f;
                if (out_bf) out_bf[pos * 16 + row] = f2bf(v);
                if (out_f32 && f32_all) out_f32[pos * 16 + row] = v;
                else if (out_f32 && row == 0) out_f32[pos] = v;
            }
        }
    }
}

// Weight and bias gradients of one layer, per block of positions:
// part_w[blk][k][out][in] = sum_pos dz[pos][out] * x[pos + off(k)][in],
// part_b[blk][out] = sum_pos dz[pos][out].
__global__ __launch_bounds__(256) void k_conv16_wgrad(ConvDims c, const uint16_t* __restrict__ x,
                                                      const uint16_t* __restrict__ dz,
                                                      float* __restrict__ part_w,
                                                      float* __restrict__ part_b) {
    __shared__ uint16_t s_x[HZ * HY * HX * 16];
    __shared__ uint16_t s_d[kTilePos * 16];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    const uint32_t blk = blockIdx.x;
    int n, z0, y0, x0;
    block_origin(c, blk, n, z0, y0, x0);
    load_halo(c, x, n, z0, y0, x0, s_x);
    for (int p = threadIdx.x; p < kTilePos; p += blockDim.x) {
        const int px = p % TX, py = (p / TX) % TY, pz = p / (TX * TY);
        const int zz = z0 + pz, yy = y0 + py, xx = x0 + px;
        uint4 lo = make_uint4(0, 0, 0, 0), hi = make_uint4(0, 0, 0, 0);
        if (zz < c.D && yy < c.H && xx < c.W) {
            const uint4* src = reinterpret_cast<const uint4*>(
                dz + ((((size_t)n * c.D + zz) * c.H + yy) * c.W + xx) * 16);
            lo = src[0];
            hi = src[1];
        }
        uint4* dst = reinterpret_cast<uint4*>(s_d + (size_t)p * 16);
        dst[0] = lo;
        dst[1] = hi;
    }
    __syncthreads();
    // wave w accumulates offsets k = w, w + 4, ... (at most 7)
    v4f acc[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) acc[j] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};
    for (int r = 0; r < TZ * TY; ++r) {
        const int zl = r / TY, yl = r % TY;
        // A operand (out x pos): dz[pos = 4*grp + i][out = row]
        v4s a;
        for (int i = 0; i < 4; ++i) a[i] = (short)s_d[(size_t)(r * TX + 4 * grp + i) * 16 + row];
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const int k = wave + 4 * j;
            if (k < 27) {
                const int dzo = k / 9 - 1, dyo = (k / 3) % 3 - 1, dxo = k % 3 - 1;
                // B operand (pos x in): x[pos + off][in = row]
                v4s bb;
                for (int i = 0; i < 4; ++i)
                    bb[i] = (short)s_x[(((size_t)(zl + 1 + dzo) * HY + (yl + 1 + dyo)) * HX +
                                        (4 * grp + i + 1 + dxo)) * 16 + row];
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[j], 0, 0, 0);
            }
        }
    }
    // acc[j][i] = D[out = 4*grp + i][in = row]
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int k = wave + 4 * j;
        if (k < 27)
            for (int i = 0; i < 4; ++i)
                part_w[(((size_t)blk * 27 + k) * 16 + 4 * grp + i) * 16 + row] = acc[j][i];
    }
    if (threadIdx.x < 16) {
        float s = 0.0f;
        for (int p = 0; p < kTilePos; ++p) s += bf2f(s_d[(size_t)p * 16 + threadIdx.x]);
        part_b[(size_t)blk * 16 + threadIdx.x] = s;
    }
}

// Sum block partials in a fixed order: out[j] = sum_b part[b][j].
__global__ void k_reduce_parts(const float* __restrict__ part, uint32_t nblk, uint32_t len,
                               float* __restrict__ out) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < len; j += gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (uint32_t b = 0; b < nblk; ++b) s += part[(size_t)b * len + j];
        out[j] = s;
    }
}

// Binary cross entropy with logits, positive weight pw, mean over n
// positions: dz (bf16, channel 0 of 16) and per-block shares of the mean loss.
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ logits,
                                             const uint8_t* __restrict__ y, uint64_t n, float pw,
                                             uint16_t* __restrict__ dz, float* __restrict__ part_loss) {
    __shared__ float s_sum[4];
    float acc = 0.0f;
    const float inv = 1.0f / (float)n;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float z = logits[i];
        const float t = y[i] ? 1.0f : 0.0f;
        const float sp_neg = fmaxf(-z, 0.0f) + log1pf(expf(-fabsf(z)));  // softplus(-z)
        const float sp_pos = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));   // softplus(z)
        acc += pw * t * sp_neg + (1.0f - t) * sp_pos;
        const float s = 1.0f / (1.0f + expf(-z));
        const float g = (s * (pw * t + 1.0f - t) - pw * t) * inv;
        uint4* o = reinterpret_cast<uint4*>(dz + i * 16);
        o[0] = make_uint4(f2bf(g), 0, 0, 0);
        o[1] = make_uint4(0, 0, 0, 0);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane_id() == 0) s_sum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part_loss[blockIdx.x] = (s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3]) * inv;
}

// Reference-layout fp32 parameters -> padded bf16 kernel weights:
// fwd[k][out][in] = W[out][in][k]; bwd[k][in][out] = W[out][in][26 - k]
// (transposed and point-reflected: the input-gradient convolution).
__global__ void k_prep_weights(const float* __restrict__ params, NetShapes s, uint16_t* __restrict__ wf,
                               uint16_t* __restrict__ wb, float* __restrict__ bias) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int layer = 0; layer < 3; ++layer) {
        const int cin = s.cin[layer], cout = s.cout[layer];
        const float* W = params + s.woff[layer];
        for (int i = tid; i < 27 * 256; i += gridDim.x * blockDim.x) {
            const int k = i / 256, a = (i / 16) % 16, b = i % 16;
            // forward: out = a, in = b
            float vf = (a < cout && b < cin) ? W[(a * cin + b) * 27 + k] : 0.0f;
            // backward: out (of the gradient conv) = in channel a, in = out channel b
            float vb = (b < cout && a < cin) ? W[(b * cin + a) * 27 + (26 - k)] : 0.0f;
            wf[(size_t)layer * 27 * 256 + i] = f2bf(vf);
            wb[(size_t)layer * 27 * 256 + i] = f2bf(vb);
        }
        if (tid < 16) bias[layer * 16 + tid] = tid < cout ? params[s.boff[layer] + tid] : 0.0f;
    }
}

// Reduced padded gradients -> reference layout.
__global__ void k_gather_grads(const float* __restrict__ gw, const float* __restrict__ gb,
                               NetShapes s, int layer, float* __restrict__ grads) {
    const int cin = s.cin[layer], cout = s.cout[layer];
    const int nw = cout * cin * 27;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nw + cout; i += gridDim.x * blockDim.x) {
        if (i < nw) {
            const int o = i / (cin * 27), ci = (i / 27) % cin, k = i % 27;
            grads[s.woff[layer] + i] = gw[((size_t)k * 16 + o) * 16 + ci];
        } else {
            grads[s.boff[layer] + (i - nw)] = gb[i - nw];
        }
    }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// ---- features and labels from the grower's state ----

// Load time: per brick-step (8^3 voxels of one timestep) min, max, mean of
// the non-NaN field values (-1 for all three when there are none).
__global__ __launch_bounds__(256) void k_brick_stats(Geom g, BrickDims bd, const float* __restrict__ f,
                                                     float4* __restrict__ stats) {
    __shared__ float s_mn[4], s_mx[4], s_sum[4], s_cnt[4];
    const uint32_t b = blockIdx.x;
    const int bx = b % bd.W, by = (b / bd.W) % bd.H, bz = (b / (bd.W * bd.H)) % bd.D,
              t = b / (bd.W * bd.H * bd.D);
    float mn = __builtin_inff(), mx = -__builtin_inff(), sum = 0.0f, cnt = 0.0f;
    for (int i = threadIdx.x; i < 512; i += blockDim.x) {
        const int x = bx * 8 + (i & 7), y = by * 8 + ((i >> 3) & 7), z = bz * 8 + (i >> 6);
        if (x < g.X && y < g.Y && z < g.Z) {
            const float v = f[(((size_t)t * g.Z + z) * g.Y + y) * g.X + x];
            if (v == v) {
                mn = fminf(mn, v);
                mx = fmaxf(mx, v);
                sum += v;
                cnt += 1.0f;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, o));
        mx = fmaxf(mx, __shfl_xor(mx, o));
        sum += __shfl_xor(sum, o);
        cnt += __shfl_xor(cnt, o);
    }
    if (lane_id() == 0) {
        s_mn[threadIdx.x >> 6] = mn;
        s_mx[threadIdx.x >> 6] = mx;
        s_sum[threadIdx.x >> 6] = sum;
        s_cnt[threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mn = fminf(fminf(s_mn[0], s_mn[1]), fminf(s_mn[2], s_mn[3]));
        mx = fmaxf(fmaxf(s_mx[0], s_mx[1]), fmaxf(s_mx[2], s_mx[3]));
        sum = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        cnt = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        stats[b] = cnt > 0 ? make_float4(mn, mx, sum / cnt, 0.0f) : make_float4(-1.f, -1.f, -1.f, 0.f);
    }
}

// Load time: particle-steps per brick-step (into stats[].w).
__global__ void k_brick_pcount(Geom g, PGeom pg, BrickDims bd, const uint32_t* __restrict__ bins,
                               float4* __restrict__ stats) {
    const uint64_t n = (uint64_t)pg.P * pg.Tpad;
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = bins[e];
        if (b == kNoVoxel) continue;
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
        const int x = tx * 32 + (b & 31), y = ty * 8 + (wi & 7), z = tz * 8 + ((wi >> 3) & 7);
        const int t = (tt << g.logBT) + (wi >> 6);
        const uint32_t bi = (((uint32_t)t * bd.D + (z >> 3)) * bd.H + (y >> 3)) * bd.W + (x >> 3);
        atomicAdd(&stats[bi].w, 1.0f);
    }
}

// Per grow: network input at brick-step (t, z, y, x): field min / max / mean
// minus the field lower bound and log1p(particle count) / 4, at t and at t-1
// (zeros at t = 0); channels 8..15 zero.
__global__ void k_features(BrickDims bd, const float4* __restrict__ stats, float f_lo,
                           uint16_t* __restrict__ x) {
    const uint64_t n = (uint64_t)bd.T * bd.D * bd.H * bd.W;
    const uint64_t per_t = (uint64_t)bd.D * bd.H * bd.W;
    const float c = (f_lo == f_lo && fabsf(f_lo) < 1e30f) ? f_lo : 0.0f;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t t = i / per_t;
        const float4 s0 = stats[i];
        const float4 s1 = t > 0 ? stats[i - per_t] : make_float4(c, c, c, 0.0f);
        uint16_t v[16];
        v[0] = f2bf(s0.x - c);
        v[1] = f2bf(s0.y - c);
        v[2] = f2bf(s0.z - c);
        v[3] = f2bf(log1pf(s0.w) * 0.25f);
        v[4] = f2bf(s1.x - c);
        v[5] = f2bf(s1.y - c);
        v[6] = f2bf(s1.z - c);
        v[7] = f2bf(log1pf(s1.w) * 0.25f);
        for (int k = 8; k < 16; ++k) v[k] = 0;
        uint4* o = reinterpret_cast<uint4*>(x + i * 16);
        o[0] = make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16), v[6] | (v[7] << 16));
        o[1] = make_uint4(0, 0, 0, 0);
    }
}

// After a grow: brick-step label = it holds a member voxel.
__global__ void k_brick_labels(Geom g, BrickDims bd, const uint32_t* __restrict__ L,
                               const uint8_t* __restrict__ active, uint8_t* __restrict__ y) {
    const uint64_t n = (uint64_t)bd.T * bd.D * bd.H * bd.W;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int bx = i % bd.W, by = (i / bd.W) % bd.H, bz = (i / ((uint64_t)bd.W * bd.H)) % bd.D;
        const int t = (int)(i / ((uint64_t)bd.W * bd.H * bd.D));
        const int tx = bx >> 2, xs = (bx & 3) * 8;  // 4 bricks of 8 x-bits per tile word
        const int tt = t >> g.logBT, tl = t & (g.BT - 1);
        const uint32_t tile = ((uint32_t)(tt * g.NZt + bz) * g.NYt + by) * g.NXt + tx;
        uint32_t any = 0;
        if (active[tile]) {
            const uint32_t* w = L + (size_t)tile * g.WPT + tl * 64;
            for (int k = 0; k < 64; ++k) any |= (w[k] >> xs) & 0xFFu;
        }
        y[i] = any ? 1 : 0;
    }
}

// Scores -> tiles to test before the rounds: a candidate tile is tested up
// front when any of its brick-steps scores at least `thr` (logit); the other
// candidates are deferred to the first sweep that reaches them.
__global__ void k_tile_predict(Geom g, BrickDims bd, const float* __restrict__ logits, float thr,
                               uint8_t* __restrict__ pred) {
    for (uint32_t tile = blockIdx.x * blockDim.x + threadIdx.x; tile < g.NT;
         tile += gridDim.x * blockDim.x) {
        uint32_t r = tile;
        const int tx = r % g.NXt;
        r /= g.NXt;
        const int ty = r % g.NYt;
        r /= g.NYt;
        const int tz = r % g.NZt;
        const int tt = r / g.NZt;
        bool hot = false;
        for (int tl = 0; tl < g.BT && !hot; ++tl) {
            const int t = (tt << g.logBT) + tl;
            if (t >= g.T) break;
            for (int k = 0; k < 4; ++k) {
                const int bx = tx * 4 + k;
                if (bx >= bd.W) break;
                const uint64_t i = (((uint64_t)t * bd.D + tz) * bd.H + ty) * bd.W + bx;
                if (logits[i] >= thr) {
                    hot = true;
                    break;
                }
            }
        }
        pred[tile] = hot ? 1 : 0;
    }
}

inline unsigned grid_for(uint64_t n, unsigned block, unsigned cap) {
    uint64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

ConvDims conv_dims(int N, int D, int H, int W) {
    ConvDims c{N, D, H, W, (W + TX - 1) / TX, (H + TY - 1) / TY, (D + TZ - 1) / TZ};
    return c;
}

}  // namespace

uint32_t nn_blocks(int N, int D, int H, int W) {
    const ConvDims c = conv_dims(N, D, H, W);
    return (uint32_t)c.N * c.nbz * c.nby * c.nbx;
}

void launch_conv16(int N, int D, int H, int W, const uint16_t* x, const uint16_t* w,
                   const float* bias, int relu, const uint16_t* mask, uint16_t* out_bf,
                   float* out_f32, hipStream_t s) {
    const ConvDims c = conv_dims(N, D, H, W);
    const uint32_t nb = nn_blocks(N, D, H, W);
    hipLaunchKernelGGL(k_conv16, dim3(grid_for(nb, 1, 8192)), dim3(256), 0, s, c, x, w, bias, relu,
                       mask, out_bf, out_f32, 0);
}

void launch_conv16_f32(int N, int D, int H, int W, const uint16_t* x, const uint16_t* w,
                       float* out_f32, hipStream_t s) {
    const ConvDims c = conv_dims(N, D, H, W);
    const uint32_t nb = nn_blocks(N, D, H, W);
    hipLaunchKernelGGL(k_conv16, dim3(grid_for(nb, 1, 8192)), dim3(256), 0, s, c, x, w,
                       (const float*)nullptr, 0, (const uint16_t*)nullptr, (uint16_t*)nullptr, out_f32, 1);
}

void launch_conv16_wgrad(int N, int D, int H, int W, const uint16_t* x, const uint16_t* dz,
                         float* part_w, float* part_b, float* gw, float* gb, hipStream_t s) {
    const ConvDims c = conv_dims(N, D, H, W);
    const uint32_t nb = nn_blocks(N, D, H, W);
    hipLaunchKernelGGL(k_conv16_wgrad, dim3(nb), dim3(256), 0, s, c, x, dz, part_w, part_b);
    hipLaunchKernelGGL(k_reduce_parts, dim3(grid_for(27 * 256, 256, 64)), dim3(256), 0, s, part_w,
                       nb, 27u * 256u, gw);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(64), 0, s, part_b, nb, 16u, gb);
}

void launch_bce(const float* logits, const uint8_t* y, uint64_t n, float pw, uint16_t* dz,
                float* part_loss, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_bce, dim3(kLossBlocks), dim3(256), 0, s, logits, y, n, pw, dz, part_loss);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(64), 0, s, part_loss, (uint32_t)kLossBlocks, 1u,
                       loss);
}

void launch_prep_weights(const float* params, const NetShapes& sh, uint16_t* wf, uint16_t* wb,
                         float* bias, hipStream_t s) {
    hipLaunchKernelGGL(k_prep_weights, dim3(27), dim3(256), 0, s, params, sh, wf, wb, bias);
}

void launch_gather_grads(const float* gw, const float* gb, const NetShapes& sh, int layer,
                         float* grads, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_grads, dim3(16), dim3(256), 0, s, gw, gb, sh, layer, grads);
}

void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                 float eps, int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n, 256, 64)), dim3(256), 0, s, p, g, m, v, n, lr, b1,
                       b2, eps, c1, c2);
}

void launch_brick_stats(const Geom& g, const PGeom& pg, const BrickDims& bd, const float* field,
                        const uint32_t* bins, float4* stats, hipStream_t s) {
    const uint32_t nb = (uint32_t)((uint64_t)bd.T * bd.D * bd.H * bd.W);
    hipLaunchKernelGGL(k_brick_stats, dim3(nb), dim3(256), 0, s, g, bd, field, stats);
    if (pg.P > 0 && bins)
        hipLaunchKernelGGL(k_brick_pcount, dim3(grid_for((uint64_t)pg.P * pg.Tpad, 256, 8192)),
                           dim3(256), 0, s, g, pg, bd, bins, stats);
}

void launch_features(const BrickDims& bd, const float4* stats, float f_lo, uint16_t* x,
                     hipStream_t s) {
    const uint64_t n = (uint64_t)bd.T * bd.D * bd.H * bd.W;
    hipLaunchKernelGGL(k_features, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, bd, stats, f_lo, x);
}

void launch_brick_labels(const Geom& g, const BrickDims& bd, const uint32_t* L,
                         const uint8_t* active, uint8_t* y, hipStream_t s) {
    const uint64_t n = (uint64_t)bd.T * bd.D * bd.H * bd.W;
    hipLaunchKernelGGL(k_brick_labels, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, g, bd, L,
                       active, y);
}

void launch_tile_predict(const Geom& g, const BrickDims& bd, const float* logits, float thr,
                         uint8_t* pred, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_predict, dim3(grid_for(g.NT, 256, 4096)), dim3(256), 0, s, g, bd,
                       logits, thr, pred);
}

}  // namespace mf4d
