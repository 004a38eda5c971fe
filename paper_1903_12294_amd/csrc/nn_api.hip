// C ABI of the brick-activity predictor network: parameters, inference,
// gradients and Adam training steps, all on the GPU.
#include <mf4d.h>

#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <new>
#include <string>

#include "nn.h"

using namespace mf4d;

struct mf4d_net {
    int device = 0;
    hipStream_t stream = nullptr;
    uint16_t* noalloc = nullptr;  // this device's copy of `scratch` (device address)
    NetShapes sh{};
    float* params = nullptr;  // fp32 masters, reference layout
    float* grads = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    uint4* wpk = nullptr;     // packed bf16 B operands: [6][kPackSlot] (forward and input
                              // gradient of each layer)
    float* bias = nullptr;    // fp32 [3][16]
    int step = 0;
    // activation buffers (grown on demand): inference (bf16 activations)
    uint64_t cap_pos = 0;
    uint16_t *a1 = nullptr, *a2 = nullptr;
    float* logits = nullptr;
    // training (fp32 activations and layer gradients)
    uint64_t cap_tpos = 0;
    uint32_t cap_blocks = 0;
    float *t1 = nullptr, *t2 = nullptr, *dz1 = nullptr, *dz2 = nullptr, *dz3 = nullptr, *tlogits = nullptr;
    float *part_w = nullptr, *part_b = nullptr, *gw = nullptr, *gb = nullptr;
    float *part_loss = nullptr, *loss = nullptr;
    float* h_loss = nullptr;
};

// Scratch of the allocation-free forward (mf4d_nn_forward_noalloc): the two
// hidden activations, bf16 [positions][16] each, for at most
// kNoAllocPositions positions: 16 MiB per GPU, held until the process ends.
// Every call on one GPU uses that GPU's copy, so calls that overlap on one
// GPU race.  Host code never passes the array's name to a kernel (on the host
// it is only a stand-in); it uses the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
constexpr uint64_t kNoAllocPositions = 1ull << 18;
static __device__ __align__(256) uint16_t scratch[2 * kNoAllocPositions * 16];

namespace {

thread_local std::string n_err;

int nfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    n_err = buf;
    return code;
}

#define NHIP(expr)                                                                            \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return nfail(e_ == hipErrorOutOfMemory ? MF4D_ERR_OOM : MF4D_ERR_HIP, "%s: %s", #expr, \
                         hipGetErrorString(e_));                                              \
    } while (0)

template <class T>
int nalloc(T** p, size_t n) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, (n ? n : 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return nfail(e == hipErrorOutOfMemory ? MF4D_ERR_OOM : MF4D_ERR_HIP, "hipMalloc failed");
    }
    return MF4D_OK;
}

template <class T>
void nfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_infer(mf4d_net* n) {
    nfree(n->a1);
    nfree(n->a2);
    nfree(n->logits);
    n->cap_pos = 0;
}

void free_train(mf4d_net* n) {
    nfree(n->t1);
    nfree(n->t2);
    nfree(n->dz1);
    nfree(n->dz2);
    nfree(n->dz3);
    nfree(n->tlogits);
    nfree(n->part_w);
    nfree(n->part_b);
    n->cap_tpos = 0;
    n->cap_blocks = 0;
}

int ensure_infer(mf4d_net* n, uint64_t pos) {
    if (pos <= n->cap_pos) return MF4D_OK;
    free_infer(n);
    int rc = nalloc(&n->a1, pos * 16);
    if (!rc) rc = nalloc(&n->a2, pos * 16);
    if (!rc) rc = nalloc(&n->logits, pos);
    if (rc) {
        free_infer(n);
        return rc;
    }
    n->cap_pos = pos;
    return MF4D_OK;
}

int ensure_train(mf4d_net* n, uint64_t pos, uint32_t blocks) {
    if (pos <= n->cap_tpos && blocks <= n->cap_blocks) return MF4D_OK;
    free_train(n);
    int rc = nalloc(&n->t1, pos * 16);
    if (!rc) rc = nalloc(&n->t2, pos * 16);
    if (!rc) rc = nalloc(&n->dz1, pos * 16);
    if (!rc) rc = nalloc(&n->dz2, pos * 16);
    if (!rc) rc = nalloc(&n->dz3, pos * 16);
    if (!rc) rc = nalloc(&n->tlogits, pos);
    if (!rc) rc = nalloc(&n->part_w, (size_t)blocks * 27 * 256);
    if (!rc) rc = nalloc(&n->part_b, (size_t)blocks * 16);
    if (rc) {
        free_train(n);
        return rc;
    }
    n->cap_tpos = pos;
    n->cap_blocks = blocks;
    return MF4D_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint16_t* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on `device` (current), looked up once.
int noalloc_scratch(int device, uint16_t** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return nfail(MF4D_ERR_UNSUPPORTED, "device index %d not below %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nfail(MF4D_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        g_scratch[device] = static_cast<uint16_t*>(ptr);
    }
    *out = g_scratch[device];
    return MF4D_OK;
}

int check_dims(int N, int D, int H, int W) {
    if (N <= 0 || D <= 0 || H <= 0 || W <= 0) return nfail(MF4D_ERR_ARG, "dims must be positive");
    if ((uint64_t)N * D * H * W >= (1ull << 31)) return nfail(MF4D_ERR_UNSUPPORTED, "too many positions");
    return MF4D_OK;
}

// Loss and gradients of every parameter (into n->grads) at training
// precision, from device x, y; dx (nullable): the input gradient.
void train_pass(mf4d_net* n, const uint16_t* x, const uint8_t* y, int N, int D, int H, int W, float pw, float* dx) {
    launch_train_forward(N, D, H, W, x, n->wpk, n->bias, n->t1, n->t2, n->tlogits, n->stream);
    launch_train_backward(N, D, H, W, x, n->wpk, n->tlogits, y, pw, n->t1, n->t2, n->dz1, n->dz2, n->dz3, dx,
                          n->part_w, n->part_b, n->gw, n->gb, n->part_loss, n->loss, n->sh, n->grads, n->stream);
}

}  // namespace

namespace mf4d {
// Inference for the grower (device pointers, the net's own stream order is
// not used: work goes on `s`).
int net_infer(mf4d_net* n, const uint16_t* x, int N, int D, int H, int W, float* logits,
              hipStream_t s) {
    int rc = check_dims(N, D, H, W);
    if (rc) return rc;
    const uint64_t pos = (uint64_t)N * D * H * W;
    rc = ensure_infer(n, pos);
    if (rc) return rc;
    launch_infer(N, D, H, W, x, n->wpk, n->bias, n->a1, n->a2, logits, s);
    return MF4D_OK;
}
const char* net_last_error() { return n_err.c_str(); }
}  // namespace mf4d

extern "C" {

int mf4d_net_num_params(void) { return net_shapes().total; }

int mf4d_net_create(mf4d_net** out, int device, void* stream) {
    if (!out) return nfail(MF4D_ERR_ARG, "out is NULL");
    *out = nullptr;
    NHIP(hipSetDevice(device));
    mf4d_net* n = new (std::nothrow) mf4d_net();
    if (!n) return nfail(MF4D_ERR_OOM, "host allocation failed");
    n->device = device;
    n->stream = (hipStream_t)stream;
    n->sh = net_shapes();
    const int P = n->sh.total;
    int rc = noalloc_scratch(device, &n->noalloc);
    if (!rc) rc = nalloc(&n->params, P);
    if (!rc) rc = nalloc(&n->grads, P);
    if (!rc) rc = nalloc(&n->m, P);
    if (!rc) rc = nalloc(&n->v, P);
    if (!rc) rc = nalloc(&n->wpk, 6 * kPackSlot);
    if (!rc) rc = nalloc(&n->bias, 48);
    if (!rc) rc = nalloc(&n->gw, 27 * 256);
    if (!rc) rc = nalloc(&n->gb, 16);
    if (!rc) rc = nalloc(&n->part_loss, kLossBlocks);
    if (!rc) rc = nalloc(&n->loss, 1);
    if (!rc && hipHostMalloc((void**)&n->h_loss, sizeof(float)) != hipSuccess)
        rc = nfail(MF4D_ERR_OOM, "pinned allocation failed");
    if (!rc) {
        launch_fill_u32((uint32_t*)n->params, 0, P, n->stream);
        launch_fill_u32((uint32_t*)n->m, 0, P, n->stream);
        launch_fill_u32((uint32_t*)n->v, 0, P, n->stream);
        launch_pack_weights(n->params, n->sh, n->wpk, n->bias, n->stream);
        if (hipStreamSynchronize(n->stream) != hipSuccess) rc = nfail(MF4D_ERR_HIP, "init failed");
    }
    if (rc) {
        mf4d_net_destroy(n);
        return rc;
    }
    *out = n;
    return MF4D_OK;
}

void mf4d_net_destroy(mf4d_net* n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    (void)hipStreamSynchronize(n->stream);
    free_infer(n);
    free_train(n);
    nfree(n->params);
    nfree(n->grads);
    nfree(n->m);
    nfree(n->v);
    nfree(n->wpk);
    nfree(n->bias);
    nfree(n->gw);
    nfree(n->gb);
    nfree(n->part_loss);
    nfree(n->loss);
    if (n->h_loss) (void)hipHostFree(n->h_loss);
    delete n;
}

const char* mf4d_net_last_error(void) { return n_err.c_str(); }

int mf4d_net_set_params(mf4d_net* n, const float* params, int where) {
    if (!n || !params) return nfail(MF4D_ERR_ARG, "NULL argument");
    NHIP(hipSetDevice(n->device));
    NHIP(hipMemcpyAsync(n->params, params, n->sh.total * sizeof(float),
                        where == MF4D_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                        n->stream));
    launch_fill_u32((uint32_t*)n->m, 0, n->sh.total, n->stream);
    launch_fill_u32((uint32_t*)n->v, 0, n->sh.total, n->stream);
    launch_pack_weights(n->params, n->sh, n->wpk, n->bias, n->stream);
    n->step = 0;
    NHIP(hipStreamSynchronize(n->stream));
    return MF4D_OK;
}

int mf4d_net_get_params(mf4d_net* n, float* params, int where) {
    if (!n || !params) return nfail(MF4D_ERR_ARG, "NULL argument");
    NHIP(hipSetDevice(n->device));
    NHIP(hipMemcpyAsync(params, n->params, n->sh.total * sizeof(float),
                        where == MF4D_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                        n->stream));
    NHIP(hipStreamSynchronize(n->stream));
    return MF4D_OK;
}

int mf4d_net_forward(mf4d_net* n, const uint16_t* x, int N, int D, int H, int W, float* logits,
                     int where) {
    if (!n || !x || !logits) return nfail(MF4D_ERR_ARG, "NULL argument");
    if (where != MF4D_DEVICE) return nfail(MF4D_ERR_ARG, "network tensors must be device pointers");
    int rc = check_dims(N, D, H, W);
    if (rc) return rc;
    NHIP(hipSetDevice(n->device));
    rc = ensure_infer(n, (uint64_t)N * D * H * W);
    if (rc) return rc;
    launch_infer(N, D, H, W, x, n->wpk, n->bias, n->a1, n->a2, logits, n->stream);
    NHIP(hipStreamSynchronize(n->stream));
    return MF4D_OK;
}

int mf4d_net_grad(mf4d_net* n, const uint16_t* x, const uint8_t* y, int N, int D, int H, int W,
                  float pos_weight, float* grads, float* loss, int where) {
    if (!n || !x || !y || !grads) return nfail(MF4D_ERR_ARG, "NULL argument");
    if (where != MF4D_DEVICE) return nfail(MF4D_ERR_ARG, "network tensors must be device pointers");
    int rc = check_dims(N, D, H, W);
    if (rc) return rc;
    NHIP(hipSetDevice(n->device));
    rc = ensure_train(n, (uint64_t)N * D * H * W, nn_blocks(N, D, H, W));
    if (rc) return rc;
    train_pass(n, x, y, N, D, H, W, pos_weight, nullptr);
    NHIP(hipMemcpyAsync(grads, n->grads, n->sh.total * sizeof(float), hipMemcpyDeviceToDevice,
                        n->stream));
    NHIP(hipMemcpyAsync(n->h_loss, n->loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NHIP(hipStreamSynchronize(n->stream));
    if (loss) *loss = *n->h_loss;
    return MF4D_OK;
}

int mf4d_net_train_step(mf4d_net* n, const uint16_t* x, const uint8_t* y, int N, int D, int H,
                        int W, float pos_weight, float lr, float* loss) {
    if (!n || !x || !y) return nfail(MF4D_ERR_ARG, "NULL argument");
    int rc = check_dims(N, D, H, W);
    if (rc) return rc;
    NHIP(hipSetDevice(n->device));
    rc = ensure_train(n, (uint64_t)N * D * H * W, nn_blocks(N, D, H, W));
    if (rc) return rc;
    train_pass(n, x, y, N, D, H, W, pos_weight, nullptr);
    n->step += 1;
    launch_adam(n->params, n->grads, n->m, n->v, n->sh.total, lr, 0.9f, 0.999f, 1e-8f, n->step,
                n->stream);
    launch_pack_weights(n->params, n->sh, n->wpk, n->bias, n->stream);
    if (loss) {
        NHIP(hipMemcpyAsync(n->h_loss, n->loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
        NHIP(hipStreamSynchronize(n->stream));
        *loss = *n->h_loss;
    }
    return MF4D_OK;
}

int mf4d_nn_forward(mf4d_net* n, const uint16_t* x, int N, int D, int H, int W, float* logits,
                    int where) {
    return mf4d_net_forward(n, x, N, D, H, W, logits, where);
}

int mf4d_nn_backward(mf4d_net* n, const uint16_t* x, const uint8_t* y, int N, int D, int H, int W,
                     float pos_weight, float* grads, float* dx, float* loss, int where) {
    if (!n || !x || !y || !grads) return nfail(MF4D_ERR_ARG, "NULL argument");
    if (where != MF4D_DEVICE) return nfail(MF4D_ERR_ARG, "network tensors must be device pointers");
    int rc = check_dims(N, D, H, W);
    if (rc) return rc;
    NHIP(hipSetDevice(n->device));
    rc = ensure_train(n, (uint64_t)N * D * H * W, nn_blocks(N, D, H, W));
    if (rc) return rc;
    train_pass(n, x, y, N, D, H, W, pos_weight, dx);
    NHIP(hipMemcpyAsync(grads, n->grads, n->sh.total * sizeof(float), hipMemcpyDeviceToDevice,
                        n->stream));
    NHIP(hipMemcpyAsync(n->h_loss, n->loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NHIP(hipStreamSynchronize(n->stream));
    if (loss) *loss = *n->h_loss;
    return MF4D_OK;
}

int mf4d_nn_forward_noalloc(mf4d_net* n, const uint16_t* x, int N, int D, int H, int W, float* logits,
                            int where) {
    if (!n || !x || !logits) return nfail(MF4D_ERR_ARG, "NULL argument");
    if (where != MF4D_DEVICE) return nfail(MF4D_ERR_ARG, "network tensors must be device pointers");
    int rc = check_dims(N, D, H, W);
    if (rc) return rc;
    const uint64_t pos = (uint64_t)N * D * H * W;
    if (pos > kNoAllocPositions)
        return nfail(MF4D_ERR_RANGE, "%llu positions exceed the %llu of the static scratch",
                     (unsigned long long)pos, (unsigned long long)kNoAllocPositions);
    if (!n->noalloc) return nfail(MF4D_ERR_STATE, "no scratch address for device %d", n->device);
    NHIP(hipSetDevice(n->device));
    launch_infer(N, D, H, W, x, n->wpk, n->bias, n->noalloc, n->noalloc + pos * 16, logits, n->stream);
    NHIP(hipGetLastError());
    return MF4D_OK;
}

int mf4d_nn_adam_step(mf4d_net* n, const float* grads, float lr, int where) {
    if (!n) return nfail(MF4D_ERR_ARG, "NULL argument");
    if (where != MF4D_DEVICE) return nfail(MF4D_ERR_ARG, "network tensors must be device pointers");
    if (!(lr == lr)) return nfail(MF4D_ERR_ARG, "lr is NaN");
    NHIP(hipSetDevice(n->device));
    if (grads && grads != n->grads)
        NHIP(hipMemcpyAsync(n->grads, grads, n->sh.total * sizeof(float), hipMemcpyDeviceToDevice,
                            n->stream));
    n->step += 1;
    launch_adam(n->params, n->grads, n->m, n->v, n->sh.total, lr, 0.9f, 0.999f, 1e-8f, n->step,
                n->stream);
    launch_pack_weights(n->params, n->sh, n->wpk, n->bias, n->stream);
    NHIP(hipStreamSynchronize(n->stream));
    return MF4D_OK;
}

}  // extern "C"
