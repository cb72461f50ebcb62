// Training and inference kernels of the envelope MLP (gfx950), behind the
// cdem_mlp_* entry points of include/cdem.h.
//
// Backward: one workgroup per 32 samples keeps the samples' activations in
// LDS and forms its partial gradient with every parameter summed over the
// samples in ascending order; a second pass sums the partials over the
// workgroups in ascending order, so a gradient is bit-reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "../../include/cdem.h"
#include "mlp_dev.h"

namespace cdem {

constexpr int kBwdSamples = 32;
constexpr int kBwdThreads = 256;
constexpr int kPartial = kMlpParams + 1;  // gradient + loss

__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ params, const float *__restrict__ f,
                                                     float *__restrict__ y, int64_t n) {
    __shared__ float P[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) P[i] = params[i];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float y0, y1;
        mlp_forward(P, f[3 * i], f[3 * i + 1], f[3 * i + 2], y0, y1);
        y[2 * i] = y0;
        y[2 * i + 1] = y1;
    }
}

// Partial gradient (and loss) of the mean pinball loss over this workgroup's samples.
__global__ void __launch_bounds__(kBwdThreads) k_mlp_backward(const float *__restrict__ params,
                                                              const float *__restrict__ f,
                                                              const float *__restrict__ target, int64_t n,
                                                              float tau, float *__restrict__ partial) {
    __shared__ float P[kMlpParams];
    __shared__ float X[kBwdSamples][3];
    __shared__ float H1[kBwdSamples][kMlpH];
    __shared__ float H2[kBwdSamples][kMlpH];
    __shared__ float DZ1[kBwdSamples][kMlpH];
    __shared__ float DZ2[kBwdSamples][kMlpH];
    __shared__ float DY[kBwdSamples][2];
    __shared__ float LOSS[kBwdSamples];
    const int tid = threadIdx.x;
    for (int i = tid; i < kMlpParams; i += blockDim.x) P[i] = params[i];
    __syncthreads();
    const int64_t s0 = (int64_t)blockIdx.x * kBwdSamples;
    const float scale = 1.0f / (2.0f * (float)n);  // mean over n samples x 2 outputs
    // phase 1: forward pass and output gradient, one thread per sample
    if (tid < kBwdSamples) {
        const int b = tid;
        const int64_t i = s0 + b;
        const bool valid = i < n;
        float x[3] = {0.f, 0.f, 0.f};
        if (valid) mlp_input(P, f[3 * i], f[3 * i + 1], f[3 * i + 2], x);
        X[b][0] = x[0]; X[b][1] = x[1]; X[b][2] = x[2];
        for (int j = 0; j < kMlpH; j++) {
            const float *w = P + kMlpOffW1 + 3 * j;
            H1[b][j] = fmaxf(P[kMlpOffB1 + j] + w[0] * x[0] + w[1] * x[1] + w[2] * x[2], 0.0f);
        }
        float y0 = P[kMlpOffB3], y1 = P[kMlpOffB3 + 1];
        for (int j = 0; j < kMlpH; j++) {
            const float *w = P + kMlpOffW2 + kMlpH * j;
            float z = P[kMlpOffB2 + j];
            for (int k = 0; k < kMlpH; k++) z = fmaf(w[k], H1[b][k], z);
            float h = fmaxf(z, 0.0f);
            H2[b][j] = h;
            y0 = fmaf(P[kMlpOffW3 + j], h, y0);
            y1 = fmaf(P[kMlpOffW3 + kMlpH + j], h, y1);
        }
        float d0 = 0.f, d1 = 0.f, l = 0.f;
        if (valid) {
            float r0 = target[2 * i] - y0, r1 = target[2 * i + 1] - y1;
            d0 = (r0 > 0.f ? -tau : 1.0f - tau) * scale;
            d1 = (r1 > 0.f ? -tau : 1.0f - tau) * scale;
            l = (fmaxf(tau * r0, (tau - 1.0f) * r0) + fmaxf(tau * r1, (tau - 1.0f) * r1)) * scale;
        }
        DY[b][0] = d0;
        DY[b][1] = d1;
        LOSS[b] = l;
        for (int j = 0; j < kMlpH; j++)
            DZ2[b][j] = H2[b][j] > 0.f ? d0 * P[kMlpOffW3 + j] + d1 * P[kMlpOffW3 + kMlpH + j] : 0.f;
    }
    __syncthreads();
    // phase 2: dz1 = relu'(z1) * W2^T dz2
    for (int idx = tid; idx < kBwdSamples * kMlpH; idx += blockDim.x) {
        int b = idx / kMlpH, i = idx % kMlpH;
        float acc = 0.f;
        if (H1[b][i] > 0.f)
            for (int j = 0; j < kMlpH; j++) acc = fmaf(P[kMlpOffW2 + kMlpH * j + i], DZ2[b][j], acc);
        DZ1[b][i] = acc;
    }
    __syncthreads();
    // phase 3: every parameter summed over the samples in ascending order
    float *out = partial + (int64_t)blockIdx.x * kPartial;
    for (int p = tid; p < kPartial; p += blockDim.x) {
        float acc = 0.f;
        if (p < kMlpOffW1) {
            acc = 0.f;  // standardisation entries are not trained
        } else if (p < kMlpOffB1) {
            int j = (p - kMlpOffW1) / 3, k = (p - kMlpOffW1) % 3;
            for (int b = 0; b < kBwdSamples; b++) acc = fmaf(DZ1[b][j], X[b][k], acc);
        } else if (p < kMlpOffW2) {
            int j = p - kMlpOffB1;
            for (int b = 0; b < kBwdSamples; b++) acc += DZ1[b][j];
        } else if (p < kMlpOffB2) {
            int j = (p - kMlpOffW2) / kMlpH, i = (p - kMlpOffW2) % kMlpH;
            for (int b = 0; b < kBwdSamples; b++) acc = fmaf(DZ2[b][j], H1[b][i], acc);
        } else if (p < kMlpOffW3) {
            int j = p - kMlpOffB2;
            for (int b = 0; b < kBwdSamples; b++) acc += DZ2[b][j];
        } else if (p < kMlpOffB3) {
            int o = (p - kMlpOffW3) / kMlpH, j = (p - kMlpOffW3) % kMlpH;
            for (int b = 0; b < kBwdSamples; b++) acc = fmaf(DY[b][o], H2[b][j], acc);
        } else if (p < kMlpParams) {
            int o = p - kMlpOffB3;
            for (int b = 0; b < kBwdSamples; b++) acc += DY[b][o];
        } else {
            for (int b = 0; b < kBwdSamples; b++) acc += LOSS[b];
        }
        out[p] = acc;
    }
}

// Sum the workgroups' partials in ascending order.
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *__restrict__ partial, int64_t nblk,
                                                    float *__restrict__ grad, float *__restrict__ loss) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kPartial) return;
    float acc = 0.f;
    for (int64_t b = 0; b < nblk; b++) acc += partial[b * kPartial + p];
    if (p < kMlpParams) grad[p] = acc;
    else if (loss) *loss = acc;
}

// Adam with bias correction; the standardisation entries stay fixed.
__global__ void __launch_bounds__(256) k_mlp_adam(float *__restrict__ params, const float *__restrict__ grad,
                                                  float *__restrict__ m, float *__restrict__ v, float lr,
                                                  float beta1, float beta2, float eps, float bc1, float bc2) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpOffW1 || p >= kMlpParams) return;
    float g = grad[p];
    float mm = beta1 * m[p] + (1.0f - beta1) * g;
    float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    params[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

}  // namespace cdem

using namespace cdem;

extern "C" int cdem_mlp_param_count(void) { return kMlpParams; }

extern "C" size_t cdem_mlp_workspace_bytes(int64_t n) {
    int64_t nblk = std::max<int64_t>(1, (n + kBwdSamples - 1) / kBwdSamples);
    return (size_t)nblk * kPartial * sizeof(float);
}

extern "C" int cdem_mlp_forward(const float *params, const float *features, float *out, int64_t n, void *stream) {
    if (!params || (n > 0 && (!features || !out)) || n < 0) return CDEM_E_INVALID;
    if (n == 0) return CDEM_OK;
    unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_mlp_forward, dim3(nb), dim3(256), 0, (hipStream_t)stream, params, features, out, n);
    return hipGetLastError() == hipSuccess ? CDEM_OK : CDEM_E_HIP;
}

extern "C" int cdem_mlp_backward(const float *params, const float *features, const float *target, int64_t n,
                                 float tau, float *grad, float *loss, void *workspace, void *stream) {
    if (!params || !features || !target || !grad || !workspace || n <= 0 || !(tau > 0.f && tau < 1.f))
        return CDEM_E_INVALID;
    int64_t nblk = (n + kBwdSamples - 1) / kBwdSamples;
    if (nblk > (int64_t)0x7fffffff) return CDEM_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_backward, dim3((unsigned)nblk), dim3(kBwdThreads), 0, st, params, features, target, n,
                       tau, (float *)workspace);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kPartial + 255) / 256), dim3(256), 0, st, (const float *)workspace, nblk,
                       grad, loss);
    return hipGetLastError() == hipSuccess ? CDEM_OK : CDEM_E_HIP;
}

// ---- allocation-free backward pass ----
// The per-workgroup partials of cdem_mlp_backward live here instead of in a
// caller workspace, for callers that cannot allocate device memory.  Every
// partial the reduction reads is first written by k_mlp_backward in the same
// call, so nothing needs clearing between calls.  One copy per device, held
// until the process ends; calls that overlap on one device share it and race.
namespace cdem {
constexpr int64_t kStaticBwdBlocks = CDEM_MLP_STATIC_MAX_SAMPLES / kBwdSamples;
__device__ __align__(256) float scratch[kStaticBwdBlocks * kPartial];
}  // namespace cdem

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_ready[kMaxDevices] = {};

// Device address of the scratch array on the current device (the host-side
// name of the array is not a device address).  Looked up once per device.
int scratch_on_current_device(float **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CDEM_E_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ready[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(cdem::scratch)) != hipSuccess || !p) return CDEM_E_HIP;
        g_scratch_ptr[dev] = (float *)p;
        g_scratch_ready[dev] = true;
    }
    *out = g_scratch_ptr[dev];
    return CDEM_OK;
}
}  // namespace

extern "C" int cdem_mlp_backward_static(const float *params, const float *features, const float *target, int64_t n,
                                        float tau, float *grad, float *loss, void *stream) {
    if (!params || !features || !target || !grad || n <= 0 || !(tau > 0.f && tau < 1.f)) return CDEM_E_INVALID;
    if (n > CDEM_MLP_STATIC_MAX_SAMPLES) return CDEM_E_INVALID;
    float *ws = nullptr;
    const int rc = scratch_on_current_device(&ws);
    if (rc != CDEM_OK) return rc;
    const int64_t nblk = (n + kBwdSamples - 1) / kBwdSamples;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_backward, dim3((unsigned)nblk), dim3(kBwdThreads), 0, st, params, features, target, n,
                       tau, ws);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kPartial + 255) / 256), dim3(256), 0, st, (const float *)ws, nblk, grad,
                       loss);
    return hipGetLastError() == hipSuccess ? CDEM_OK : CDEM_E_HIP;
}

extern "C" int cdem_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t t, float lr, float beta1,
                             float beta2, float eps, void *stream) {
    if (!params || !grad || !m || !v || t < 1 || !(lr > 0.f)) return CDEM_E_INVALID;
    float bc1 = 1.0f - powf(beta1, (float)t), bc2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad,
                       m, v, lr, beta1, beta2, eps, bc1, bc2);
    return hipGetLastError() == hipSuccess ? CDEM_OK : CDEM_E_HIP;
}
