// Host-side state of a learned-collide network (struct lb_mlp of the C ABI):
// device pointers into the caller's workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mlp_common.hpp"

struct lb_mlp {
    hipStream_t stream;
    char* ws;
    size_t bytes;
    int32_t max_batch;
    int32_t max_wg;       // max_batch / samples per training workgroup
    float* params;        // packed FP32 master parameters
    float* adam_m;
    float* adam_v;
    uint16_t* W1b;
    uint16_t* W2b;
    uint16_t* W3b;
    uint16_t* W2t;
    uint16_t* W3t;
    uint16_t* W2p;
    uint16_t* W3p;
    // FP8 form of the hidden layer (Net): scaled copies, made from params
    uint16_t* W1s;
    uint8_t* W2q;
    uint16_t* W3s;
    float* b1s;
    float* b2s;
    float* gk2;
    int32_t precision;    // LB_MLP_F16 or LB_MLP_FP8
    float* norm;          // [4][64]
    float* fnorm;         // [4][64], folded from norm for inference (Net::fnorm)
    float* partials;      // [max_wg][NPARAM_PAD]
    double* lossp;        // [max_wg]
    double* loss_epoch;   // [MAX_EPOCHS][2]: sum, count
    double* stats;        // [STAT_BLOCKS][74] and means [74]
    float* grad;          // [NPARAM_PAD]
    int64_t adam_t;       // Adam steps taken
    char err[512];

    d2q37::mlp::Net net() const
    {
        d2q37::mlp::Net n;
        n.W1b = W1b;
        n.W2b = W2b;
        n.W3b = W3b;
        n.W2t = W2t;
        n.W3t = W3t;
        n.W2p = W2p;
        n.W3p = W3p;
        n.W1s = W1s;
        n.W2q = W2q;
        n.W3s = W3s;
        n.b1s = b1s;
        n.b2s = b2s;
        n.gk2 = gk2;
        n.params = params;
        n.norm = norm;
        n.fnorm = fnorm;
        return n;
    }
};

namespace d2q37 {
namespace mlp {
constexpr int NPARAM_PAD = (NPARAM + 63) / 64 * 64;
constexpr int TRAIN_SAMPLES = 32;  // samples per training workgroup
constexpr int MAX_EPOCHS = 4096;
constexpr int STAT_BLOCKS = 512;
constexpr int NSTAT = 2 * Q;  // z features then y features
}  // namespace mlp
}  // namespace d2q37
