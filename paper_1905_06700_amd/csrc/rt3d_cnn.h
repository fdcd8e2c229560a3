// rt3d_cnn.h -- shapes and buffers of the learned depth denoiser (internal).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "rt3d_dev.h"

namespace rt3d {

constexpr int CNN_LAYERS = 4;
constexpr double CNN_GATE = 3.0;   // neighbour depth gate of the features, in sigma_h
// master (trained) channel counts and the counts stored for the matrix cores
constexpr int CNN_CIN[CNN_LAYERS] = {16, 32, 32, 32};
constexpr int CNN_COUT[CNN_LAYERS] = {32, 32, 32, 3};
constexpr int CNN_CIS[CNN_LAYERS] = {16, 32, 32, 32};
constexpr int CNN_COS[CNN_LAYERS] = {32, 32, 32, 16};
// offsets of each layer in the flat master vector ([3][3][cin][cout] then bias)
constexpr int CNN_L0 = 9 * 16 * 32 + 32, CNN_L1 = 9 * 32 * 32 + 32;
constexpr int CNN_OFF[CNN_LAYERS] = {0, CNN_L0, CNN_L0 + CNN_L1, CNN_L0 + 2 * CNN_L1};
constexpr int CNN_PARAMS = (9 * 16 * 32 + 32) + 2 * (9 * 32 * 32 + 32) + (9 * 32 * 3 + 3);

struct CnnWeights {
    float* master = nullptr;        // FP32 master weights [CNN_PARAMS]
    float* m = nullptr;             // Adam first moment
    float* v = nullptr;             // Adam second moment
    __half* wt[CNN_LAYERS] = {};    // forward layout [cos][9 * cis]
    __half* wb[CNN_LAYERS] = {};    // backward-data layout [cis][9 * cos] (layers 1..3)
    float* bias[CNN_LAYERS] = {};   // [cos]
    long long step = 0;
};

struct CnnBuffers {
    __half* act[5] = {};            // features [P][16], three hidden [P][32], output [P][16]
    __half* dy16 = nullptr;         // output gradient [P][16]
    __half* dA = nullptr;           // hidden gradients [P][32]
    __half* dB = nullptr;
    float* tgt = nullptr;           // [3][P]
    uint8_t* msk = nullptr;         // [3][P]
    float* lpart = nullptr;         // loss partials [2 * blocks]
    float* part = nullptr;          // weight-gradient partials [groups][9 * 32][32]
    float* bpart = nullptr;         // bias-gradient partials [groups][32]
    float* grad = nullptr;          // flat gradient [CNN_PARAMS]
};

struct CnnAdam {
    float lr, beta1, beta2, eps;
};

unsigned cnn_wgrad_groups(const Shape& sh);
hipError_t launch_cnn_prepare(const CnnWeights& w, hipStream_t st);
hipError_t launch_cnn_forward(const Shape& sh, DevState s, float sigma_h, const CnnWeights& w, const CnnBuffers& b,
                              hipStream_t st);
// The same network output as launch_cnn_forward, by the fused kernel (no
// stored activations: inference only).
hipError_t launch_cnn_infer(const Shape& sh, DevState s, float sigma_h, const CnnWeights& w, const CnnBuffers& b,
                            hipStream_t st);
hipError_t launch_cnn_apply(const Shape& sh, const CnnBuffers& b, float sigma_h, double tmax, DevState s,
                            hipStream_t st);
hipError_t launch_cnn_unpack(const Shape& sh, const CnnBuffers& b, float* out, hipStream_t st);
hipError_t launch_cnn_train_step(const Shape& sh, DevState s, float sigma_h, const float* truth, int S,
                                 CnnWeights& w, const CnnBuffers& b, const CnnAdam& opt, float* loss,
                                 hipStream_t st);

}  // namespace rt3d
