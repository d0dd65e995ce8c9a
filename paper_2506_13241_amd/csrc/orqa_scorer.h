// Learned truncation scorer: shared declarations (kernels and host engine).
#pragma once

#include "orqa_device.h"

namespace orqa {

constexpr int kScIn = 160;   // features per string
constexpr int kScH = 128;    // hidden width
constexpr int kScThreads = 512;  // forward workgroup: 8 waves sharing one copy of the weights
// flat fp32 parameter vector: W1 (128x160) | b1 (128) | W2 (128x128) | b2 (128) | W3 (128) | b3 (1)
constexpr int kScOffW1 = 0;
constexpr int kScOffB1 = kScOffW1 + kScH * kScIn;
constexpr int kScOffW2 = kScOffB1 + kScH;
constexpr int kScOffB2 = kScOffW2 + kScH * kScH;
constexpr int kScOffW3 = kScOffB2 + kScH;
constexpr int kScOffB3 = kScOffW3 + kScH;
constexpr int kScParams = kScOffB3 + 1;  // 37249

// Device copy of the network used by the kernels: bf16 weights, fp32 biases,
// and the feature definition (qubit mask, letter, scale per feature).
struct ScorerDev {
    uint16_t* W1;  // 128 x 160
    uint16_t* W2;  // 128 x 128
    uint16_t* W3;  // 128
    float* b1;
    float* b2;
    float* b3;
    ulonglong2* qmask;  // 160
    uint8_t* letter;    // 160: 0 X, 1 Y, 2 Z, 3 any
    float* fscale;      // 160
};

__device__ __forceinline__ uint16_t scorer_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ void scorer_store_param(const ScorerDev& net, int i, float v) {
    if (i < kScOffB1) net.W1[i - kScOffW1] = scorer_bf16(v);
    else if (i < kScOffW2) net.b1[i - kScOffB1] = v;
    else if (i < kScOffB2) net.W2[i - kScOffW2] = scorer_bf16(v);
    else if (i < kScOffW3) net.b2[i - kScOffB2] = v;
    else if (i < kScOffB3) net.W3[i - kScOffW3] = scorer_bf16(v);
    else net.b3[0] = v;
}

struct ScorerFwdArgs {
    ScorerDev net;
    const ulonglong2* X;  // keys (virtual front/back array when nf_ptr is set)
    const ulonglong2* Z;
    uint64_t n;           // used when nf_ptr is null
    const uint64_t* nf_ptr;
    const uint64_t* nb_ptr;
    uint64_t cap;
    int xrot, nq;
    float* y_out;         // n (log10 of the predicted weight)
    float* z1_out;        // n x 128 or null
    float* z2_out;        // n x 128 or null
    uint16_t* f_out;      // n x 160 or null
    uint64_t* counters;   // [0] strings scored, [1] launches (added by workgroup 0), or null
};

struct ScorerBwdArgs {
    ScorerDev net;
    uint64_t n;
    const float* y;
    const float* target;
    const float* z1;
    const float* z2;
    float* dy;   // n
    float* dz1;  // n x 128
    float* dz2;  // n x 128
};

hipError_t launch_scorer_forward(const ScorerFwdArgs& a, hipStream_t s, int grid);
hipError_t launch_scorer_backward(const ScorerBwdArgs& a, const uint16_t* f, float* grad, hipStream_t s);
hipError_t launch_scorer_loss(const float* y, const float* t, uint64_t n, double* out, hipStream_t s);
hipError_t launch_scorer_adam(float* p, const float* g, float* m, float* v, int n, float lr, int step,
                              const ScorerDev& net, hipStream_t s);
hipError_t launch_scorer_set(const float* p, int n, const ScorerDev& net, hipStream_t s);

}  // namespace orqa
