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

const char* net_last_error();
uint32_t nn_blocks(int N, int D, int H, int W);
void launch_conv16(int N, int D, int H, int W, const uint16_t* x, const uint16_t* w,
                   const float* bias, int relu, const uint16_t* mask, uint16_t* out_bf,
                   float* out_f32, hipStream_t s);
// The convolution without bias or activation, all 16 output channels as
// fp32 [..][16] (the input gradient of the first layer).
void launch_conv16_f32(int N, int D, int H, int W, const uint16_t* x, const uint16_t* w,
                       float* out_f32, hipStream_t s);
void launch_conv16_wgrad(int N, int D, int H, int W, const uint16_t* x, const uint16_t* dz,
                         float* part_w, float* part_b, float* gw, float* gb, hipStream_t s);
void launch_bce(const float* logits, const uint8_t* y, uint64_t n, float pw, uint16_t* dz,
                float* part_loss, float* loss, hipStream_t s);
void launch_prep_weights(const float* params, const NetShapes& sh, uint16_t* wf, uint16_t* wb,
                         float* bias, hipStream_t s);
void launch_gather_grads(const float* gw, const float* gb, const NetShapes& sh, int layer,
                         float* grads, hipStream_t s);
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
