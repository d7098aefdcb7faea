// Device interface of the message-passing network kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace twk {

constexpr int MpnnFeat = 4;                                // [1, deg/8, core/8, n/64]
constexpr int MpnnLayerParams = 2 * 64 * 64 + 64;          // Ws, Wn, b
constexpr int MpnnParams = 3 * MpnnLayerParams + 2 * 128 + 2;  // + Wo, bo

struct MpnnArgs {
    const uint64_t *adj;     // [graphs][64] adjacency rows
    const float *feat;       // [graphs][64][MpnnFeat]
    const int32_t *n;        // [graphs]
    const float *params;     // fp32 master parameters (biases and heads read from here)
    const uint16_t *wsb, *wsbt, *wnb, *wnbt;  // bf16 weights [3][64][64], [out][in] and [in][out]
    const float *targets;    // [graphs][2] or nullptr
    float grad_scale;        // d(loss)/dy = 2 (y - t) * grad_scale
    float *pred;             // [graphs][2] or nullptr
    float *sq_err;           // [graphs][2] or nullptr
    float *grads;            // [graphs][MpnnParams] per-graph gradients, or nullptr (inference)
    float *trace;            // [graphs][MpnnTraceFloats] float32 intermediates (test hook), or nullptr
};

// Trace layout (floats, per graph; every 64 x 64 block row-major [node][feature]):
//   M_l  = A H_l before its bfloat16 rounding       l = 0..2   at MpnnTrM + l * 4096
//   Z_l  = H_l Ws^T + M_l Wn^T + b before the ReLU  l = 0..2   at MpnnTrZ + l * 4096
//   r [128], y [2]                                             at MpnnTrR
//   dH_3 (gradient of the loss with respect to H_3)            at MpnnTrDH3
//   dZ_l before its bfloat16 rounding               l = 0..2   at MpnnTrDZ + l * 4096
//   P_l = dZ_l Wn_l before its bfloat16 rounding    l = 1, 2   at MpnnTrP + (l - 1) * 4096
//   dH_l = dZ_l Ws_l + A P_l                        l = 1, 2   at MpnnTrDH + (l - 1) * 4096
constexpr int MpnnTrM = 0;
constexpr int MpnnTrZ = 3 * 4096;
constexpr int MpnnTrR = 6 * 4096;
constexpr int MpnnTrDH3 = MpnnTrR + 256;
constexpr int MpnnTrDZ = MpnnTrDH3 + 4096;
constexpr int MpnnTrP = MpnnTrDZ + 3 * 4096;
constexpr int MpnnTrDH = MpnnTrP + 2 * 4096;
constexpr int MpnnTraceFloats = MpnnTrDH + 2 * 4096;

struct MpnnOptArgs {
    float *params, *m, *v;
    const float *grads;
    float lr, beta1, beta2, eps, weight_decay;
    float bc1, bc2;          // 1 - beta^t bias corrections
};

size_t mpnn_smem_bytes();
hipError_t launch_mpnn(const MpnnArgs &a, int graphs, hipStream_t s);
hipError_t launch_mpnn_reduce(const float *partial, int graphs, float *grads, hipStream_t s);
hipError_t launch_mpnn_adamw(const MpnnOptArgs &o, hipStream_t s);
hipError_t launch_mpnn_pack(const float *params, uint16_t *wsb, uint16_t *wsbt, uint16_t *wnb, uint16_t *wnbt,
                            hipStream_t s);

}  // namespace twk
