// Brick-activity predictor: a 3-layer 3D convolutional network over the grid of
// 8^3-voxel bricks of each timestep, trained on the grower's own results and
// used by the learned scheduler (score order of the tiles, which candidate
// tiles are tested before the rounds).
//
// Activations are channels-last [N][D][H][W][16].  A layer is a 3x3x3
// convolution with zero padding on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16): for 16 input channels one instruction takes two
// kernel offsets x 16 channels (14 per output tile of 16 positions x 16
// channels, the last half empty); the first layer reads only its 8 real
// input channels, four offsets x 8 channels per instruction (7 per tile).
// Weights are bf16, accumulation fp32.
//
// Two precisions of the activations:
//   inference (the scheduler's scores): bf16 activations, one bf16 operand;
//   training (gradients): fp32 activations and fp32 layer gradients.  A
//   convolution splits each fp32 operand into three bf16 pieces (all 24
//   significant bits), so its pre-activations, and the ReLU decisions taken
//   on them, are as accurate as fp32 arithmetic; a weight gradient splits
//   both operands into high part and remainder (hi*hi + hi*lo + lo*hi, about
//   16 bits).  The gradients then follow the fp64 reference element by
//   element.
// The input-gradient of a layer is the same convolution with transposed,
// point-reflected weights; the weight gradient is a reduction over positions
// on the same matrix cores, per block, then summed in a fixed order
// (deterministic).  Parameters are fp32 masters updated by Adam.
#include "nn.h"

namespace mf4d {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
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

__device__ __forceinline__ v4f mfma(const uint4& a, const uint4& b, v4f acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   acc, 0, 0, 0);
}

__device__ __forceinline__ uint4 pack8(const uint16_t* h) {
    return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// Eight fp32 values -> bf16 high parts and bf16 remainders (v - hi, exact in
// fp32, then rounded): about 16 significant bits.
__device__ __forceinline__ void split8(const float* v, uint4& hi, uint4& lo) {
    uint16_t h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = f2bf(v[e]);
        l[e] = f2bf(v[e] - bf2f(h[e]));
    }
    hi = pack8(h);
    lo = pack8(l);
}

// The same in three pieces (the remainder split once more): all 24
// significant bits of an fp32 value, so that a convolution of these operands
// with fp32 accumulation is as accurate as fp32 arithmetic.
__device__ __forceinline__ void split8x3(const float* v, uint4& hi, uint4& mid, uint4& lo) {
    uint16_t h[8], m[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = f2bf(v[e]);
        const float r = v[e] - bf2f(h[e]);
        m[e] = f2bf(r);
        l[e] = f2bf(r - bf2f(m[e]));
    }
    hi = pack8(h);
    mid = pack8(m);
    lo = pack8(l);
}

constexpr int TX = 16, TY = 4, TZ = 4;                  // output positions per block
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;   // with halo
constexpr int kHalo = HX * HY * HZ;                    // 648
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

// Kernel offset k = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1).
__device__ __forceinline__ int halo_shift(int k) {
    const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
    return (dz * HY + dy) * HX + dx;
}

// Stage the (TZ+2)(TY+2)(TX+2)-position input tile, CIN channels of each
// position (of the 16 stored), zero outside the grid.  T = uint16_t (bf16) or
// float.
template <int CIN, class T>
__device__ void load_halo(const ConvDims& c, const T* __restrict__ x, int n, int z0, int y0, int x0,
                          T* s_x) {
    constexpr int kVec = CIN * (int)sizeof(T) / 16;  // 16-byte pieces per position
    for (int i = threadIdx.x; i < kHalo * kVec; i += blockDim.x) {
        const int p = i / kVec, v = i % kVec;
        const int hx = p % HX, hy = (p / HX) % HY, hz = p / (HX * HY);
        const int zz = z0 + hz - 1, yy = y0 + hy - 1, xx = x0 + hx - 1;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (zz >= 0 && zz < c.D && yy >= 0 && yy < c.H && xx >= 0 && xx < c.W)
            val = reinterpret_cast<const uint4*>(x + ((((size_t)n * c.D + zz) * c.H + yy) * c.W + xx) * 16)[v];
        reinterpret_cast<uint4*>(s_x + (size_t)p * CIN)[v] = val;
    }
}

// Instructions per 16 x 16 output tile: two offsets x 16 channels or four
// offsets x 8 channels each.
template <int CIN>
constexpr int ksteps() { return CIN == 16 ? 14 : 7; }

// (kernel offset, first channel) of the operand lane group g takes in step j;
// offset 27 does not exist (that part of the operand is zero).
template <int CIN>
__device__ __forceinline__ void step_part(int j, int g, int& k, int& c0) {
    if (CIN == 16) {
        k = 2 * j + (g >> 1);
        c0 = 8 * (g & 1);
    } else {
        k = 4 * j + g;
        c0 = 0;
    }
}

enum ConvOut : int { OUT_BF16 = 0, OUT_F32 = 1, OUT_LOGIT = 2 };

// out = conv(x, w) + bias, optionally ReLU, optionally zero where mask <= 0
// (mask: the layer's forward activation, fp32 [..][16]: the ReLU derivative).
// x: T [..][16], CIN channels read; F32 inputs are split into two bf16
// operands.  wpk: packed B operands, [ksteps][64 lanes] x 16 bytes.  Output
// OUT_BF16: bf16 [..][16]; OUT_F32: fp32 [..][16]; OUT_LOGIT: channel 0 as
// fp32 [N][D][H][W].
template <int CIN, class T, int OUT>
__global__ __launch_bounds__(256) void k_conv(ConvDims c, const T* __restrict__ x, const uint4* __restrict__ wpk,
                                              const float* __restrict__ bias, int relu,
                                              const float* __restrict__ mask, void* __restrict__ out) {
    constexpr bool kF32 = sizeof(T) == 4;
    constexpr int NK = ksteps<CIN>();
    __shared__ T s_x[kHalo * CIN];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    uint4 bw[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) bw[j] = wpk[j * 64 + lane];
    const float b = bias ? bias[row] : 0.0f;
    const uint32_t nblocks = (uint32_t)c.N * c.nbz * c.nby * c.nbx;
    for (uint32_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        int n, z0, y0, x0;
        block_origin(c, blk, n, z0, y0, x0);
        __syncthreads();
        load_halo<CIN>(c, x, n, z0, y0, x0, s_x);
        __syncthreads();
        for (int r = wave; r < TZ * TY; r += 4) {
            const int zl = r / TY, yl = r % TY;
            const int base = ((zl + 1) * HY + (yl + 1)) * HX + (row + 1);
            v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int j = 0; j < NK; ++j) {
                int k, c0;
                step_part<CIN>(j, grp, k, c0);
                const int p = base + halo_shift(k < 27 ? k : 26);
                if (kF32) {
                    float v[8];
                    const float4* src = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(s_x) +
                                                                        (size_t)p * CIN + c0);
                    const float4 u0 = src[0], u1 = src[1];
                    v[0] = u0.x; v[1] = u0.y; v[2] = u0.z; v[3] = u0.w;
                    v[4] = u1.x; v[5] = u1.y; v[6] = u1.z; v[7] = u1.w;
                    uint4 hi, mid, lo;
                    split8x3(v, hi, mid, lo);
                    if (k >= 27) hi = mid = lo = make_uint4(0, 0, 0, 0);
                    acc = mfma(hi, bw[j], acc);
                    acc = mfma(mid, bw[j], acc);
                    acc = mfma(lo, bw[j], acc);
                } else {
                    uint4 a = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(s_x) +
                                                             (size_t)p * CIN + c0);
                    if (k >= 27) a = make_uint4(0, 0, 0, 0);
                    acc = mfma(a, bw[j], acc);
                }
            }
            // acc[i] = D[position x0 + 4*grp + i][output channel row]
            const int z = z0 + zl, y = y0 + yl;
            if (z >= c.D || y >= c.H) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int xx = x0 + 4 * grp + i;
                if (xx >= c.W) continue;
                const size_t pos = (((size_t)n * c.D + z) * c.H + y) * c.W + xx;
                float v = acc[i] + b;
                if (relu) v = fmaxf(v, 0.0f);
                if (mask && !(mask[pos * 16 + row] > 0.0f)) v = 0.0f;
                if (OUT == OUT_BF16) static_cast<uint16_t*>(out)[pos * 16 + row] = f2bf(v);
                else if (OUT == OUT_F32) static_cast<float*>(out)[pos * 16 + row] = v;
                else if (row == 0) static_cast<float*>(out)[pos] = v;
            }
        }
    }
}

// Weight and bias gradients of one layer, per block of positions:
// part_w[blk][k][out][in] = sum_pos dz[pos][out] * x[pos + off(k)][in],
// part_b[blk][out] = sum_pos dz[pos][out].  dz: fp32 [..][16] (COUT channels
// real); x: T [..][16], CIN channels read.  Positions are the reduction axis:
// one instruction takes 32 positions (two rows of the tile); each fp32
// operand is split into bf16 high part and remainder.
template <int CIN, class T>
__global__ __launch_bounds__(256) void k_wgrad(ConvDims c, const T* __restrict__ x, const float* __restrict__ dz,
                                               float* __restrict__ part_w, float* __restrict__ part_b) {
    constexpr bool kF32 = sizeof(T) == 4;
    __shared__ T s_x[kHalo * CIN];
    __shared__ float s_d[kTilePos * 16];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    const uint32_t blk = blockIdx.x;
    int n, z0, y0, x0;
    block_origin(c, blk, n, z0, y0, x0);
    load_halo<CIN>(c, x, n, z0, y0, x0, s_x);
    for (int i = threadIdx.x; i < kTilePos * 4; i += blockDim.x) {
        const int p = i >> 2, v = i & 3;
        const int px = p % TX, py = (p / TX) % TY, pz = p / (TX * TY);
        const int zz = z0 + pz, yy = y0 + py, xx = x0 + px;
        float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
        if (zz < c.D && yy < c.H && xx < c.W)
            val = reinterpret_cast<const float4*>(dz + ((((size_t)n * c.D + zz) * c.H + yy) * c.W + xx) * 16)[v];
        reinterpret_cast<float4*>(s_d + (size_t)p * 16)[v] = val;
    }
    __syncthreads();
    // wave w accumulates offsets k = w, w + 4, ... (at most 7)
    v4f acc[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) acc[j] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};
    for (int ch = 0; ch < kTilePos / 32; ++ch) {
        // positions q = 32 ch + 8 grp + e: rows 2 ch + (q >> 4) & 1, x = q & 15
        float dv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) dv[e] = s_d[(size_t)(32 * ch + 8 * grp + e) * 16 + row];
        uint4 ahi, alo;
        split8(dv, ahi, alo);
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const int k = wave + 4 * j;
            if (k >= 27) continue;
            const int sh = halo_shift(k);
            uint4 bhi, blo = make_uint4(0, 0, 0, 0);
            if (row < CIN) {
                if (kF32) {
                    float xv[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int q = 32 * ch + 8 * grp + e;
                        const int r = q >> 4, px = q & 15, zl = r / TY, yl = r % TY;
                        const int p = ((zl + 1) * HY + (yl + 1)) * HX + (px + 1) + sh;
                        xv[e] = reinterpret_cast<const float*>(s_x)[(size_t)p * CIN + row];
                    }
                    split8(xv, bhi, blo);
                } else {
                    uint16_t h[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int q = 32 * ch + 8 * grp + e;
                        const int r = q >> 4, px = q & 15, zl = r / TY, yl = r % TY;
                        const int p = ((zl + 1) * HY + (yl + 1)) * HX + (px + 1) + sh;
                        h[e] = reinterpret_cast<const uint16_t*>(s_x)[(size_t)p * CIN + row];
                    }
                    bhi = pack8(h);
                }
            } else {
                bhi = make_uint4(0, 0, 0, 0);
            }
            acc[j] = mfma(ahi, bhi, acc[j]);
            acc[j] = mfma(alo, bhi, acc[j]);
            if (kF32) acc[j] = mfma(ahi, blo, acc[j]);
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
        for (int p = 0; p < kTilePos; ++p) s += s_d[(size_t)p * 16 + threadIdx.x];
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
// positions: dz (fp32 [..][16], channel 0; the rest zero) and per-block
// shares of the mean loss.
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ logits,
                                             const uint8_t* __restrict__ y, uint64_t n, float pw,
                                             float* __restrict__ dz, float* __restrict__ part_loss) {
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
        float4* o = reinterpret_cast<float4*>(dz + i * 16);
        o[0] = make_float4(g, 0.f, 0.f, 0.f);
        o[1] = o[2] = o[3] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane_id() == 0) s_sum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part_loss[blockIdx.x] = (s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3]) * inv;
}

// fp32 parameters (reference layout) -> packed bf16 B operands and biases.
// Forward of layer l (input channels cin_l): B[kappa][out], kappa = (offset,
// input channel) in the order step_part gives.  Input gradient of layer l: the
// convolution of the layer's output gradient (cout_l channels, read as 16, or
// as 8 when cout_l = 1) with W[out][in][26 - k] transposed.
// Slot s: 0..2 forward of layers 0..2, 3..5 input gradient of layers 0..2.
__global__ void k_pack_weights(const float* __restrict__ params, NetShapes sh, uint4* __restrict__ wpk,
                               float* __restrict__ bias) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = tid; i < 6 * kPackSlot; i += gridDim.x * blockDim.x) {
        const int slot = i / kPackSlot, r = i % kPackSlot;
        const int j = r / 64, lane = r % 64, g = lane >> 4, col = lane & 15;
        const int layer = slot % 3;
        const bool bwd = slot >= 3;
        const int cin = sh.cin[layer], cout = sh.cout[layer];
        const float* W = params + sh.woff[layer];
        // channels the operand reads on its input side
        const int cread = bwd ? (cout == 1 ? 8 : 16) : (cin == 8 ? 8 : 16);
        const int nk = cread == 16 ? 14 : 7;
        uint16_t h[8];
        for (int e = 0; e < 8; ++e) {
            float v = 0.0f;
            if (j < nk) {
                const int k = cread == 16 ? 2 * j + (g >> 1) : 4 * j + g;
                const int ci = (cread == 16 ? 8 * (g & 1) : 0) + e;
                if (k < 27) {
                    if (!bwd && col < cout && ci < cin) v = W[(col * cin + ci) * 27 + k];
                    if (bwd && col < cin && ci < cout) v = W[(ci * cin + col) * 27 + (26 - k)];
                }
            }
            h[e] = f2bf(v);
        }
        wpk[i] = pack8(h);
    }
    for (int i = tid; i < 48; i += gridDim.x * blockDim.x) {
        const int layer = i / 16, o = i % 16;
        bias[i] = o < sh.cout[layer] ? params[sh.boff[layer] + o] : 0.0f;
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

template <int CIN, class T, int OUT>
void conv_launch(int N, int D, int H, int W, const T* x, const uint4* wpk, const float* bias, int relu,
                 const float* mask, void* out, hipStream_t s) {
    const ConvDims c = conv_dims(N, D, H, W);
    const uint32_t nb = (uint32_t)c.N * c.nbz * c.nby * c.nbx;
    hipLaunchKernelGGL((k_conv<CIN, T, OUT>), dim3(grid_for(nb, 1, 8192)), dim3(256), 0, s, c, x, wpk, bias, relu,
                       mask, out);
}

template <int CIN, class T>
void wgrad_launch(int N, int D, int H, int W, const T* x, const float* dz, float* part_w, float* part_b, float* gw,
                  float* gb, hipStream_t s) {
    const ConvDims c = conv_dims(N, D, H, W);
    const uint32_t nb = (uint32_t)c.N * c.nbz * c.nby * c.nbx;
    hipLaunchKernelGGL((k_wgrad<CIN, T>), dim3(nb), dim3(256), 0, s, c, x, dz, part_w, part_b);
    hipLaunchKernelGGL(k_reduce_parts, dim3(grid_for(27 * 256, 256, 64)), dim3(256), 0, s, part_w, nb, 27u * 256u,
                       gw);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(64), 0, s, part_b, nb, 16u, gb);
}

}  // namespace

uint32_t nn_blocks(int N, int D, int H, int W) {
    const ConvDims c = conv_dims(N, D, H, W);
    return (uint32_t)c.N * c.nbz * c.nby * c.nbx;
}

void launch_infer(int N, int D, int H, int W, const uint16_t* x, const uint4* wpk, const float* bias,
                  uint16_t* a1, uint16_t* a2, float* logits, hipStream_t s) {
    conv_launch<8, uint16_t, OUT_BF16>(N, D, H, W, x, wpk + 0 * kPackSlot, bias, 1, nullptr, a1, s);
    conv_launch<16, uint16_t, OUT_BF16>(N, D, H, W, a1, wpk + 1 * kPackSlot, bias + 16, 1, nullptr, a2, s);
    conv_launch<16, uint16_t, OUT_LOGIT>(N, D, H, W, a2, wpk + 2 * kPackSlot, bias + 32, 0, nullptr, logits, s);
}

void launch_train_forward(int N, int D, int H, int W, const uint16_t* x, const uint4* wpk, const float* bias,
                          float* a1, float* a2, float* logits, hipStream_t s) {
    conv_launch<8, uint16_t, OUT_F32>(N, D, H, W, x, wpk + 0 * kPackSlot, bias, 1, nullptr, a1, s);
    conv_launch<16, float, OUT_F32>(N, D, H, W, a1, wpk + 1 * kPackSlot, bias + 16, 1, nullptr, a2, s);
    conv_launch<16, float, OUT_LOGIT>(N, D, H, W, a2, wpk + 2 * kPackSlot, bias + 32, 0, nullptr, logits, s);
}

void launch_train_backward(int N, int D, int H, int W, const uint16_t* x, const uint4* wpk, const float* logits,
                           const uint8_t* y, float pw, const float* a1, const float* a2, float* dz1, float* dz2,
                           float* dz3, float* dx, float* part_w, float* part_b, float* gw, float* gb,
                           float* part_loss, float* loss, const NetShapes& sh, float* grads, hipStream_t s) {
    const uint64_t pos = (uint64_t)N * D * H * W;
    hipLaunchKernelGGL(k_bce, dim3(kLossBlocks), dim3(256), 0, s, logits, y, pos, pw, dz3, part_loss);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(64), 0, s, part_loss, (uint32_t)kLossBlocks, 1u, loss);
    // layer 3: weights from a2 and dz3; dz2 = input gradient masked by relu'(z2)
    wgrad_launch<16, float>(N, D, H, W, a2, dz3, part_w, part_b, gw, gb, s);
    hipLaunchKernelGGL(k_gather_grads, dim3(16), dim3(256), 0, s, gw, gb, sh, 2, grads);
    conv_launch<8, float, OUT_F32>(N, D, H, W, dz3, wpk + 5 * kPackSlot, nullptr, 0, a2, dz2, s);
    // layer 2
    wgrad_launch<16, float>(N, D, H, W, a1, dz2, part_w, part_b, gw, gb, s);
    hipLaunchKernelGGL(k_gather_grads, dim3(16), dim3(256), 0, s, gw, gb, sh, 1, grads);
    conv_launch<16, float, OUT_F32>(N, D, H, W, dz2, wpk + 4 * kPackSlot, nullptr, 0, a1, dz1, s);
    // layer 1: weights from the bf16 inputs; the input gradient on request
    wgrad_launch<8, uint16_t>(N, D, H, W, x, dz1, part_w, part_b, gw, gb, s);
    hipLaunchKernelGGL(k_gather_grads, dim3(16), dim3(256), 0, s, gw, gb, sh, 0, grads);
    if (dx) conv_launch<16, float, OUT_F32>(N, D, H, W, dz1, wpk + 3 * kPackSlot, nullptr, 0, nullptr, dx, s);
}

void launch_pack_weights(const float* params, const NetShapes& sh, uint4* wpk, float* bias, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_weights, dim3(21), dim3(256), 0, s, params, sh, wpk, bias);
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
