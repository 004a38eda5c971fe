// Internal declarations of the brick-activity predictor (nn.hip).
#pragma once

#include "mf4d_internal.h"

namespace mf4d {

// Parameter layout (fp32, the reference layout): for each layer l,
// W_l [cout][cin][3][3][3] at woff[l], then b_l [cout] at boff[l].
struct NetShapes {
    int cin[3], cout[3];
    int woff[3], boff[3];
    int total;
};

inline NetShapes net_shapes() {
    NetShapes s{};
    const int ci[3] = {8, 16, 16}, co[3] = {16, 16, 1};
    int off = 0;
    for (int l = 0; l < 3; ++l) {
        s.cin[l] = ci[l];
        s.cout[l] = co[l];
        s.woff[l] = off;
        off += co[l] * ci[l] * 27;
        s.boff[l] = off;
        off += co[l];
    }
    s.total = off;
    return s;
}

// Brick grid: 8^3 voxels of one timestep per brick.
struct BrickDims {
    int T, D, H, W;
};

constexpr int kLossBlocks = 256;
// Packed B operands of one convolution: up to 14 instruction steps x 64 lanes,
// 16 bytes (8 bf16) each.
constexpr int kPackSlot = 14 * 64;

const char* net_last_error();
uint32_t nn_blocks(int N, int D, int H, int W);
// Inference: bf16 activations a1, a2 ([pos][16]), logits fp32 [pos].  x: bf16
// [pos][16] (channels 0..7 read).  wpk: [6][kPackSlot] packed weights.
void launch_infer(int N, int D, int H, int W, const uint16_t* x, const uint4* wpk, const float* bias,
                  uint16_t* a1, uint16_t* a2, float* logits, hipStream_t s);
// Training forward: fp32 activations a1, a2 ([pos][16]) and logits.
void launch_train_forward(int N, int D, int H, int W, const uint16_t* x, const uint4* wpk, const float* bias,
                          float* a1, float* a2, float* logits, hipStream_t s);
// Loss (mean BCE, positive weight pw, into *loss on the device), layer
// gradients dz1..dz3 (fp32 [pos][16]), every parameter's gradient into grads
// (reference layout), and with dx non-null the input gradient (fp32
// [pos][16]).  part_w / part_b: per-block partials (nn_blocks of them).
void launch_train_backward(int N, int D, int H, int W, const uint16_t* x, const uint4* wpk, const float* logits,
                           const uint8_t* y, float pw, const float* a1, const float* a2, float* dz1, float* dz2,
                           float* dz3, float* dx, float* part_w, float* part_b, float* gw, float* gb,
                           float* part_loss, float* loss, const NetShapes& sh, float* grads, hipStream_t s);
// fp32 parameters -> packed bf16 operands (forward and input gradient of each
// layer) and biases [3][16].
void launch_pack_weights(const float* params, const NetShapes& sh, uint4* wpk, float* bias, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                 float eps, int step, hipStream_t s);
void launch_brick_stats(const Geom& g, const PGeom& pg, const BrickDims& bd, const float* field,
                        const uint32_t* bins, float4* stats, hipStream_t s);
void launch_features(const BrickDims& bd, const float4* stats, float f_lo, uint16_t* x,
                     hipStream_t s);
void launch_brick_labels(const Geom& g, const BrickDims& bd, const uint32_t* L,
                         const uint8_t* active, uint8_t* y, hipStream_t s);
void launch_tile_predict(const Geom& g, const BrickDims& bd, const float* logits, float thr,
                         uint8_t* pred, hipStream_t s);

}  // namespace mf4d
