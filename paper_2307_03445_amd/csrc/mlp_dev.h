// Envelope MLP of the learned detection interval: device-side definitions
// shared by the MLP kernels and the detection chain of libcdem.
//
// Per bin: raw features f = (max sphere speed, max sphere acceleration,
// occupancy) -> u = (log(f0 + 1e-6), log(f1 + 1e-3), log(1 + f2)) ->
// x = (u - mu) / sigma -> 64 ReLU -> 64 ReLU -> (log speed envelope,
// log acceleration envelope).  FP32 arithmetic on the vector ALUs: at
// 3 -> 64 -> 64 -> 2 per bin there is no dense contraction worth a matrix core.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdem {

constexpr int kMlpH = 64;
constexpr int kMlpOffMu = 0, kMlpOffSig = 3, kMlpOffW1 = 6;
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpH * 3;
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpH;
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpH * kMlpH;
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpH;
constexpr int kMlpOffB3 = kMlpOffW3 + 2 * kMlpH;
constexpr int kMlpParams = kMlpOffB3 + 2;  // 4552

__device__ __forceinline__ void mlp_input(const float *P, float f0, float f1, float f2, float *x) {
    float u0 = logf(f0 + 1e-6f), u1 = logf(f1 + 1e-3f), u2 = log1pf(f2);
    x[0] = (u0 - P[kMlpOffMu]) / P[kMlpOffSig];
    x[1] = (u1 - P[kMlpOffMu + 1]) / P[kMlpOffSig + 1];
    x[2] = (u2 - P[kMlpOffMu + 2]) / P[kMlpOffSig + 2];
}

// Forward pass with the parameters P (usually staged in LDS).
__device__ __forceinline__ void mlp_forward(const float *P, float f0, float f1, float f2, float &y0, float &y1) {
    float x[3];
    mlp_input(P, f0, f1, f2, x);
    float h1[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; j++) {
        const float *w = P + kMlpOffW1 + 3 * j;
        float z = P[kMlpOffB1 + j] + w[0] * x[0] + w[1] * x[1] + w[2] * x[2];
        h1[j] = fmaxf(z, 0.0f);
    }
    float a0 = P[kMlpOffB3], a1 = P[kMlpOffB3 + 1];
    for (int j = 0; j < kMlpH; j++) {
        const float *w = P + kMlpOffW2 + kMlpH * j;
        float z = P[kMlpOffB2 + j];
#pragma unroll
        for (int i = 0; i < kMlpH; i++) z = fmaf(w[i], h1[i], z);
        float h = fmaxf(z, 0.0f);
        a0 = fmaf(P[kMlpOffW3 + j], h, a0);
        a1 = fmaf(P[kMlpOffW3 + kMlpH + j], h, a1);
    }
    y0 = a0;
    y1 = a1;
}

// The same forward pass with the second layer's weights transposed (Wt[i][j]
// = W2[j][i], staged so by the caller): the first layer is evaluated one unit
// at a time and spread over all 64 accumulators of the second, which keeps
// the registers at the 64 accumulators.  Every sum is taken in the same order
// as in mlp_forward, so the results are identical.
__device__ __forceinline__ void mlp_forward_t(const float *P, const float *Wt, float f0, float f1, float f2, float &y0,
                                              float &y1) {
    float x[3];
    mlp_input(P, f0, f1, f2, x);
    float z[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; j++) z[j] = P[kMlpOffB2 + j];
#pragma unroll 1
    for (int i = 0; i < kMlpH; i++) {
        const float *w = P + kMlpOffW1 + 3 * i;
        const float h = fmaxf(P[kMlpOffB1 + i] + w[0] * x[0] + w[1] * x[1] + w[2] * x[2], 0.0f);
        const float4 *wr = (const float4 *)(Wt + kMlpH * i);
#pragma unroll
        for (int j4 = 0; j4 < kMlpH / 4; j4++) {
            const float4 q = wr[j4];
            z[4 * j4] = fmaf(q.x, h, z[4 * j4]);
            z[4 * j4 + 1] = fmaf(q.y, h, z[4 * j4 + 1]);
            z[4 * j4 + 2] = fmaf(q.z, h, z[4 * j4 + 2]);
            z[4 * j4 + 3] = fmaf(q.w, h, z[4 * j4 + 3]);
        }
    }
    float a0 = P[kMlpOffB3], a1 = P[kMlpOffB3 + 1];
#pragma unroll
    for (int j = 0; j < kMlpH; j++) {
        const float h = fmaxf(z[j], 0.0f);
        a0 = fmaf(P[kMlpOffW3 + j], h, a0);
        a1 = fmaf(P[kMlpOffW3 + kMlpH + j], h, a1);
    }
    y0 = a0;
    y1 = a1;
}

}  // namespace cdem
